"""Build-time check of the compiled kernels: no workgroup barrier inside a
loop that lanes leave one by one.

In the gfx950 assembly, a loop whose exit depends on per-lane values keeps
the lanes that have left parked (removed from exec with
`s_andn2_b64 exec, exec, <exit mask>`) until every lane has left.  If such a
loop holds an `s_barrier`, the lanes still inside can meet the other waves at
the barrier without the parked ones: in a persistent kernel whose loop head
is "thread 0 takes the next query from the queue, barrier, everyone reads
it", a per-query early exit compiled this way sends every lane but thread 0
back to the barrier to re-read the same slot for ever.  The kernels are
written so that this cannot happen (no early exit from a loop body that
holds barriers, loop-control values in scalar registers); this module checks
the compiled code for it, loop by loop, using the loop annotations the
compiler writes into its assembly.

Usage: python -m paper_2206_13574_amd.asm_check [source.hip ...]
(default: every .hip source of the library); exits 1 if a kernel is flagged.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile
from collections import defaultdict

from . import build as _build

_LOOP_EXIT = re.compile(r"s_andn2_b64 exec, exec, s\[")


def _functions(text: str):
    name, cur = None, []
    for line in text.splitlines():
        m = re.match(r"^(_Z\S+):", line)
        if m:
            name, cur = m.group(1), []
            continue
        if name is None:
            continue
        cur.append(line)
        if line.startswith(".Lfunc_end"):
            yield name, cur
            name = None


def _blocks(lines):
    """Basic blocks with their loop: the header of the innermost loop they
    belong to, whether they are that header, and (for a header) the
    enclosing loops.  The compiler writes a nested loop's header as a label
    line naming the outermost parent, comment lines naming the other
    parents, then "This Inner Loop Header"."""
    out, cur = [], None
    for line in lines:
        m = re.match(r"^(\.LBB\d+_\d+|; %bb\.\d+):(.*)$", line)
        if m:
            if cur:
                out.append(cur)
            lab = m.group(1).replace("; %bb.", "bb.")
            cur = {"lab": lab, "loop": None, "parents": [], "text": [], "header": False, "code": False}
            note = m.group(2)
            mm = re.search(r"in Loop: Header=(BB\d+_\d+)", note)
            if mm:
                cur["loop"] = mm.group(1)
            mm = re.search(r"Parent Loop (BB\d+_\d+)", note)
            if mm:
                cur["parents"].append(mm.group(1))
            if "Loop Header" in note:
                cur["header"] = True
                cur["loop"] = lab.lstrip(".").replace("LBB", "BB")
        elif cur is not None:
            if not cur["code"] and line.lstrip().startswith(";"):
                mm = re.search(r"Parent Loop (BB\d+_\d+)", line)
                if mm:
                    cur["parents"].append(mm.group(1))
                elif "Loop Header" in line:
                    cur["header"] = True
                    cur["loop"] = cur["lab"].lstrip(".").replace("LBB", "BB")
            elif line.strip():
                cur["code"] = True
            cur["text"].append(line)
    if cur:
        out.append(cur)
    return out


def flagged_loops(lines) -> list:
    """Loop headers whose loop (with nested loops) holds an s_barrier and
    whose own blocks remove exiting lanes from exec."""
    own, every, parent = defaultdict(list), defaultdict(list), {}
    for b in _blocks(lines):
        if not b["loop"]:
            continue
        own[b["loop"]].append(b)
        every[b["loop"]].append(b)
        if b["header"]:
            parent[b["loop"]] = b["parents"][-1] if b["parents"] else None
    for h in list(own):
        p = parent.get(h)
        while p:
            every[p].extend(own[h])
            p = parent.get(p)
    out = []
    for h in own:
        barrier = any("s_barrier" in t for b in every[h] for t in b["text"])
        lane_exit = any(_LOOP_EXIT.search(t) for b in own[h] for t in b["text"])
        if barrier and lane_exit:
            out.append(h)
    return out


def lane_loops(lines) -> list:
    """Loops that step through the active lanes of a wave one at a time
    (find the first lane of a mask, read that lane's value, clear the lane):
    the form the compiler's atomic optimizer gives an atomic whose address is
    the same in every lane and whose value is not, before one atomic from
    one lane.  Returns [(header, nesting depth)], depth 1 for an outermost
    loop.  Inside the per-entry loops such a loop costs several instructions
    per active lane for every entry."""
    own, depth = defaultdict(list), {}
    for b in _blocks(lines):
        if not b["loop"]:
            continue
        own[b["loop"]].append(b)
        if b["header"]:
            depth[b["loop"]] = len(b["parents"]) + 1
    out = []
    for h, bs in own.items():
        text = [t for b in bs for t in b["text"]]
        if any("s_ff1_i32_b64" in t for t in text) and any("v_readlane_b32" in t for t in text):
            out.append((h, depth.get(h, 1)))
    return out


def check_asm(text: str) -> dict:
    """{kernel symbol: [flagged loop headers]} for every function in `text`."""
    return {name: flagged_loops(lines) for name, lines in _functions(text)}


def device_asm(src: str) -> str:
    """gfx950 assembly of one HIP source, with the library's flags."""
    pkg = os.path.dirname(os.path.abspath(__file__))
    inc = ["-I", os.path.join(os.path.dirname(pkg), "include"), "-I", os.path.join(pkg, "csrc")]
    flags = [f for f in _build.HIP_FLAGS if f not in ("-fPIC",)]
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "k.s")
        r = subprocess.run(["hipcc"] + flags + inc + ["--cuda-device-only", "-S", "-o", out, src],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(r.stdout + r.stderr)
        with open(out) as f:
            return f.read()


def main(argv=None) -> int:
    srcs = (argv if argv else [s for s in _build.sources() if s.endswith(".hip")])
    bad = 0
    for src in srcs:
        for name, loops in check_asm(device_asm(src)).items():
            if loops:
                bad += 1
                print(f"{os.path.basename(src)}: {name}: barrier in a lane-exit loop at {loops}")
    print("barrier check:", "FAILED" if bad else "ok", f"({len(srcs)} sources)")
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
