"""Pruning report: exact Gwfa against the heuristic of Algorithm 4 (a sweep of
a_diff) and the learned keep/drop network (a sweep of keep thresholds, plus
an untrained network and keep-all weights) on one GPU.

For every mode: query bases aligned per second (device time of the alignment
launch, queries resident and packed), speedup over exact, the fraction of
reads whose distance exceeds the exact one, the mean excess over all reads
and over the exceeding reads, and the wavefront work relative to exact.
Prints one JSON line per mode and a Markdown table.

Usage: python -m paper_2206_13574_amd.eval_prune --workload cfg3 [--reads N]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import gwfa, synth, train_prune, tune

WORKLOADS = {"cfg1": synth.cfg1, "cfg2": synth.cfg2, "cfg3": synth.cfg3, "cfg4": synth.cfg4,
             "cfg4b": lambda: synth.cfg4(sparse=True)}


def log(msg):
    print(f"[eval] {msg}", file=sys.stderr, flush=True)


def timed(ctx, graph, batch, out, o, repeats: int):
    torch = ctx.torch
    ms = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        gwfa.align_dev(ctx, graph, batch, out, o)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    res, _, _ = gwfa.fetch(out, batch.n)
    return float(np.median(ms)), res


def run_baselines(ctx, W, gate, period, run):
    """The untrained network (same shape and scales, calibrated threshold) and
    keep-all weights."""
    rng = np.random.default_rng(4242)
    w0 = train_prune.init_params(rng)
    ctx.mlp_load(train_prune.to_bf16_bits(w0), W["scale"])
    run("untrained network", gwfa.opts(prune=gwfa.PRUNE_LEARNED, keep_threshold=W["tau"], mlp_gate=gate,
                                       mlp_period=period, traceback=False), "calibrated tau")
    keep_all = np.zeros(gwfa.MLP_N, dtype=np.uint16)
    keep_all[gwfa.MLP_N - 1] = 0x4120   # b3 = 10: every logit is 10
    ctx.mlp_load(keep_all, W["scale"])
    run("keep-all network", gwfa.opts(prune=gwfa.PRUNE_LEARNED, keep_threshold=0.0, mlp_gate=gate,
                                      mlp_period=period, traceback=False))



def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="cfg3", choices=sorted(WORKLOADS))
    ap.add_argument("--reads", type=int, default=None, help="first N reads of the workload")
    ap.add_argument("--weights", default=train_prune.DEFAULT_PATH)
    ap.add_argument("--taus", default="auto", help="comma list, or auto (around the calibrated threshold)")
    ap.add_argument("--a-diffs", default="25,50,100,200,400,1000,20000")
    ap.add_argument("--gate", type=int, default=None)
    ap.add_argument("--period", type=int, default=None)
    ap.add_argument("--repeats", type=int, default=1)
    ap.add_argument("--lanes", type=int, default=None, help="lanes per query (default: the tuned configuration)")
    ap.add_argument("--lanes-heuristic", type=int, default=None,
                    help="lanes per query of the Algorithm 4 runs (default: the measured ones, else --lanes)")
    ap.add_argument("--lanes-learned", type=int, default=None,
                    help="lanes per query of the network runs (default: the measured ones, else --lanes)")
    ap.add_argument("--json", default=None, help="also write the rows to this file")
    ap.add_argument("--no-baselines", action="store_true",
                    help="skip the untrained and keep-all networks (each about as slow as exact or slower)")
    a = ap.parse_args(argv)

    import torch
    t0 = time.time()
    g, r = WORKLOADS[a.workload]()
    if a.reads:
        r = r.subset(np.arange(min(a.reads, r.n)))
    bases = int(r.off[-1])
    log(f"{a.workload}: {r.n} reads, {bases} bases, {g.n_vtx} V ({time.time() - t0:.1f} s)")
    stream = torch.cuda.Stream(device=torch.device("cuda", 0))
    ctx = gwfa.Context(0, stream=stream)
    cfg = tune.best_config(a.workload)
    if a.lanes:
        cfg["lanes"] = a.lanes
    ctx.config(**cfg)
    log(f"launch configuration {cfg}")
    graph = gwfa.Graph.of(ctx, g)
    with torch.cuda.stream(stream):
        batch = gwfa.upload_reads(ctx, r.seq, r.off, r.v_start)
        out = gwfa.alloc_out(ctx, r.n, 0)
    gwfa.pack_dev(ctx, batch, out.err)
    torch.cuda.synchronize()

    W = train_prune.load(a.weights)
    gate = W["gate"] if a.gate is None else a.gate
    period = W["period"] if a.period is None else a.period
    rows = []
    cur = {"lanes": cfg["lanes"]}

    def run(mode, o, note=""):
        ctx.stats(reset=True)
        ms, res = timed(ctx, graph, batch, out, o, a.repeats)
        st = ctx.stats(reset=True)
        rows.append(dict(mode=mode, note=note, ms=ms, res=res, lanes=cur["lanes"], mlp=st["mlp_evals"] / a.repeats,
                         pruned=st["pruned"] / a.repeats))
        log(f"{mode:28s} {ms:10.1f} ms  {note}")
        return res

    exact = run("exact", gwfa.opts(traceback=False))
    lanes_h = a.lanes_heuristic or (a.lanes if a.lanes else tune.best_lanes(a.workload, "heuristic"))
    lanes_l = a.lanes_learned or (a.lanes if a.lanes else tune.best_lanes(a.workload, "learned"))
    def reconfigure(lanes, o):
        # new working memory is allocated (and cleared) by the first launch
        # after a configuration change: one untimed launch takes that cost
        ctx.config(**dict(cfg, lanes=lanes))
        cur["lanes"] = lanes
        gwfa.align_dev(ctx, graph, batch, out, o)
        torch.cuda.synchronize()

    reconfigure(lanes_h, gwfa.opts(prune=gwfa.PRUNE_HEURISTIC, a_diff=50, traceback=False))
    log(f"Algorithm 4 runs at {lanes_h} lanes per query")
    for ad in [int(x) for x in a.a_diffs.split(",") if x]:
        run(f"heuristic a_diff={ad}", gwfa.opts(prune=gwfa.PRUNE_HEURISTIC, a_diff=ad, traceback=False))
    ctx.mlp_load(W["w_bf16"], W["scale"])
    reconfigure(lanes_l, gwfa.opts(prune=gwfa.PRUNE_LEARNED, keep_threshold=W["tau"], mlp_gate=gate,
                                   mlp_period=period, traceback=False))
    log(f"network runs at {lanes_l} lanes per query")
    taus = ([W["tau"] + d for d in (-4.0, -2.0, -1.0, 0.0, 1.0, 2.0, 4.0)] if a.taus == "auto"
            else [float(x) for x in a.taus.split(",")])
    for tau in taus:
        run(f"learned tau={tau:+.3f}", gwfa.opts(prune=gwfa.PRUNE_LEARNED, keep_threshold=tau, mlp_gate=gate,
                                                 mlp_period=period, traceback=False),
            "calibrated" if abs(tau - W["tau"]) < 1e-6 else "")
    if not a.no_baselines:
        run_baselines(ctx, W, gate, period, run)

    t_ex = rows[0]["ms"]
    w_ex = float(exact["work"].sum())
    table = []
    for row in rows:
        res = row.pop("res")
        ok = (res["status"] == 0) & (exact["status"] == 0)
        exc = (res["dist"] - exact["dist"])[ok]
        if (exc < 0).any():
            raise RuntimeError(f"{row['mode']}: a distance below the exact one")
        over = exc > 0
        row.update(bases_per_s=bases / (row["ms"] / 1000.0), speedup=t_ex / row["ms"],
                   frac_over=float(over.mean()) if len(exc) else 0.0, mean_excess=float(exc.mean()) if len(exc) else 0.0,
                   mean_excess_over=float(exc[over].mean()) if over.any() else 0.0,
                   work_vs_exact=float(res["work"].sum()) / w_ex, not_ok=int((~ok).sum()), reads=r.n,
                   workload=a.workload, gate=gate, period=period)
        table.append(row)
        print(json.dumps(row), flush=True)
    print("\n| mode | lanes | ms | bases/s | speedup | reads over | mean excess | excess (over) | work/exact | MLP evals |")
    print("|---|---|---|---|---|---|---|---|---|---|")
    for t in table:
        print(f"| {t['mode']} {t['note']} | {t['lanes']} | {t['ms']:.1f} | {t['bases_per_s']:.3e} | {t['speedup']:.2f} | "
              f"{t['frac_over']:.4f} | {t['mean_excess']:.3f} | {t['mean_excess_over']:.2f} | "
              f"{t['work_vs_exact']:.3f} | {t['mlp']:.3g} |")
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(table, fh, indent=1)
    graph.close()
    ctx.close()


if __name__ == "__main__":
    main()
