"""Writes the expected results of every read of the full-size workloads
(cfg2: 20,000 reads on the 1 Mb DAG; cfg3: 2,000 x 100 kb reads on the
cyclic 500 kb graph; cfg4: 50,000 reads on the 10 Mb bubble graph) with the
value-capped form of Eq. 1 (oracle/, orc_dp_batch): values saturated at D+1
with D the read's injected edit count, which bounds the distance from above
because the generating walk aligns the read with that many edits; the result
is exact whenever the distance is <= D, and a saturated read is an error.

Calls only oracle/ and the seeded input generator (synth).  Output:
tests/golden/<workload>.npz with dist, end_v, end_off (int32, one per read)
and the SHA-256 of the generated inputs, so that a test can tell when the
generator no longer makes the same reads.

Usage: python tests/golden/make_full_size.py cfg2 [cfg3 cfg4] [--threads N]
"""
import argparse
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2206_13574_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def input_hash(g, r) -> str:
    h = hashlib.sha256()
    for a in (g.seq, g.seg_off, g.edge_src, g.edge_dst, r.seq, r.off, r.v_start, r.n_edits):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def workload(name):
    return {"cfg2": synth.cfg2, "cfg3": synth.cfg3, "cfg4": synth.cfg4}[name]()


def run(name, threads, chunk):
    t0 = time.time()
    g, r = workload(name)
    digest = input_hash(g, r)
    print(f"[{name}] {r.n} reads, {int(r.off[-1])} bases, graph {g.n_vtx} V ({time.time() - t0:.0f} s)", flush=True)
    out = np.zeros((r.n, 3), dtype=np.int32)
    # longest reads first inside each chunk keeps the threads busy
    order = np.argsort(-(r.off[1:] - r.off[:-1]), kind="stable")
    t1 = time.time()
    for c0 in range(0, r.n, chunk):
        idx = order[c0:c0 + chunk]
        sub = r.subset(idx)
        res = O.dp_batch(g, sub.seq, sub.off, sub.v_start, sub.n_edits, n_threads=threads)
        if (res[:, 0] < 0).any():
            bad = idx[res[:, 0] < 0]
            raise SystemExit(f"[{name}] reads {bad[:10].tolist()} saturated at their injected edit count")
        out[idx] = res
        done = min(c0 + chunk, r.n)
        print(f"[{name}] {done}/{r.n} reads, {time.time() - t1:.0f} s", flush=True)
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, dist=out[:, 0], end_v=out[:, 1], end_off=out[:, 2],
                        input_sha256=np.array(digest), threads=np.array(threads),
                        seconds=np.array(time.time() - t1))
    print(f"[{name}] wrote {path} ({time.time() - t1:.0f} s of oracle time)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="+", choices=["cfg2", "cfg3", "cfg4"])
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=500)
    a = ap.parse_args()
    for w in a.workloads:
        run(w, a.threads, a.chunk)


if __name__ == "__main__":
    main()
