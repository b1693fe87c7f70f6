"""Keep-threshold calibration of the trained pruning network for one
workload shape, on held-out graphs and reads of that shape.

The threshold stored with the weights was chosen on held-out graphs of the
training shape (5 kb bubble graphs, 1 kb reads) from a grid of 19 logit
quantiles; when even the largest of them leaves no read above its exact
distance, the grid says nothing about more aggressive thresholds.  This tool
evaluates that grid plus thresholds above it (steps of `--step` up to
`--hi`) on held-out sets of a named shape, exact and learned runs both made
by the library, and keeps the largest threshold whose runs leave at most
`--target` of the reads above their exact distance.  The result goes to
prune_tau.json under the shape's name, with the whole table; the benchmark
uses it for workloads of that shape.

Shapes: "cfg2" (the 1 Mb DAG with lognormal 10 kb reads; graph seeds
2201, 2202, ..., read seeds 2301, ...: none of them is the benchmark's).

Usage: python -m paper_2206_13574_amd.calibrate_prune --shape cfg2
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import gwfa, synth, train_prune

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "prune_tau.json")


def held_out(shape: str, n_graphs: int, n_reads: int):
    if shape == "cfg2":
        return [synth.cfg2_shaped(2201 + k, 2301 + k, n_reads) for k in range(n_graphs)], \
            dict(graph_seeds=[2201 + k for k in range(n_graphs)], read_seeds=[2301 + k for k in range(n_graphs)])
    raise ValueError(f"unknown shape {shape!r}")


def load(path: str = DEFAULT_PATH) -> dict:
    """Per-shape thresholds ({} when none has been calibrated)."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--shape", default="cfg2")
    ap.add_argument("--graphs", type=int, default=2)
    ap.add_argument("--reads", type=int, default=1000, help="reads per held-out graph")
    ap.add_argument("--target", type=float, default=0.005, help="largest fraction of reads over exact")
    ap.add_argument("--step", type=float, default=0.5)
    ap.add_argument("--hi", type=float, default=12.0)
    ap.add_argument("--out", default=DEFAULT_PATH)
    a = ap.parse_args(argv)
    t0 = time.time()
    W = train_prune.load()
    grid = sorted({round(float(c["tau"]), 3) for c in W["meta"]["calib"]} | {round(W["tau"], 3)})
    grid += [round(x, 3) for x in np.arange(grid[-1] + a.step, a.hi + 1e-9, a.step)]
    sets, seeds = held_out(a.shape, a.graphs, a.reads)
    ctx = gwfa.Context(0)
    over = np.zeros(len(grid))
    work = np.zeros(len(grid))
    n_reads = work_exact = 0
    try:
        ctx.mlp_load(W["w_bf16"], W["scale"])
        for g, r in sets:
            graph = gwfa.Graph.of(ctx, g)
            ex, _ = gwfa.align(ctx, graph, r.seq, r.off, r.v_start, gwfa.opts(traceback=False))
            if (ex["status"] != gwfa.ST_OK).any():
                raise RuntimeError("an exact run did not finish")
            n_reads += r.n
            work_exact += int(ex["work"].sum())
            for t, tau in enumerate(grid):
                lr_, _ = gwfa.align(ctx, graph, r.seq, r.off, r.v_start,
                                    gwfa.opts(prune=gwfa.PRUNE_LEARNED, keep_threshold=float(tau), mlp_gate=W["gate"],
                                              mlp_period=W["period"], traceback=False))
                fin = lr_["status"] == gwfa.ST_OK
                if (fin & (lr_["dist"] < ex["dist"])).any():
                    raise RuntimeError("a pruned run went below the exact distance")
                over[t] += int((~fin | (lr_["dist"] > ex["dist"])).sum())   # unfinished counts as over
                work[t] += int(lr_["work"].sum())
            graph.close()
    finally:
        ctx.close()
    over /= max(n_reads, 1)
    work /= max(work_exact, 1)
    for t, o, wk in zip(grid, over, work):
        print(f"tau {t:+.3f}: reads over exact {o:.4f}, work vs exact {wk:.3f}", flush=True)
    ok = [t for t, o in zip(grid, over) if o <= a.target]
    tau = max(ok) if ok else min(grid)
    print(f"chosen tau {tau:+.3f} for {a.shape}", flush=True)
    table = load(a.out)
    table[a.shape] = dict(tau=tau, target=a.target, gate=W["gate"], period=W["period"], reads=a.graphs * a.reads,
                          **seeds, grid=[dict(tau=t, over=float(o), work=float(wk)) for t, o, wk in zip(grid, over, work)],
                          seconds=round(time.time() - t0, 1))
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"wrote {a.out}", flush=True)


if __name__ == "__main__":
    main()
