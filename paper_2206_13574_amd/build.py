"""Builds the HIP library (libgwfa.so) for gfx950 with hipcc, in-tree."""
import os
import subprocess
import sys

_PKG = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_PKG)
LIB = os.path.join(_PKG, "libgwfa.so")

# Packed FP32 instructions are kept off in every HIP object.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def sources():
    c = os.path.join(_PKG, "csrc")
    return [os.path.join(c, f) for f in sorted(os.listdir(c)) if f.endswith((".hip", ".cpp"))]


def build(verbose: bool = False) -> str:
    inc = ["-I", os.path.join(_ROOT, "include"), "-I", os.path.join(_PKG, "csrc")]
    tmp = LIB + ".tmp"
    cmd = ["hipcc"] + HIP_FLAGS + inc + ["-shared", "-o", tmp] + sources()
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    if verbose and (r.stdout or r.stderr):
        # the host pass warns that it does not know the packed-fp32 feature
        lines = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
        if lines:
            print("\n".join(lines))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
