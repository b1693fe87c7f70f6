#!/usr/bin/env python3
"""Benchmark: query bases aligned per second on one MI355X.

One step = the whole path over one batch with the queries already resident
in HBM: ASCII -> 2-bit packing of every query on the device, then exact
graph wavefront alignment of the batch (screen pass, extension, crossings,
end test, expansion, walk traceback) in one persistent-kernel launch.

Default workload: the largest configuration, 50,000 reads of 10-30 kb
(per-read error 1-10%) against a 10 Mb bubble graph (SNP every ~100 bp,
indel 1-20 bp every ~500 bp; synthetic, seeded); the 1 Mb DAG with 20,000
lognormal reads is measured after it as a secondary figure.  Prints ONE
JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes (bytes the method must move, independent of this
# implementation's layout): per wavefront entry, read the entry (12 B: v, k,
# offset), probe and update its diagonal record (8 B) and write the next
# entry (12 B); per 32-base compare chunk, one query and one label word
# (16 B), at least one chunk per entry; per admitted crossing, the out-edge
# range and target (12 B) plus the new entry (12 B).  With traceback each
# entry also reads and writes its trace index (4 + 4 B) and each crossing
# pushes a trace record (8 B) and its de-duplication key (8 B), Algorithm 5.
B_ENTRY, B_CHUNK, B_CROSS = 32, 16, 24
B_ENTRY_TB, B_PUSH = 8, 16


WORKLOADS = {
    "cfg2": "1 Mb DAG (SNP/1 kb, indel 1-50 bp/5 kb, SV 1-10 kb/100 kb), 20k reads lognormal median 10 kb "
            "clipped 1-50 kb, error U(0.1%,5%)",
    "cfg1": "5 kb DAG (SNP/100 bp, indel 1-20 bp/500 bp), 50 reads x 1 kb, 1% error",
    "cfg3": "500 kb backbone with 200 tandem-repeat self-loops (unit 10-200 bp), 2k reads x 100 kb, 1-30 laps, "
            "1% error",
    "cfg4": "10 Mb DAG at cfg1 densities, 50k reads U(10-30 kb), error U(1%,10%)",
}


def make_workload(name, n_reads=None):
    from paper_2206_13574_amd import synth
    if name == "cfg1":
        return synth.cfg1()
    if name == "cfg2":
        return synth.cfg2(n_reads or 20000)
    if name == "cfg3":
        return synth.cfg3(n_reads or 2000)
    if name == "cfg4":
        return synth.cfg4(n_reads or 50000)
    raise SystemExit(f"unknown workload {name}")


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo, as lscpu shows it)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(g, r, order, threads, seconds):
    import oracle as O
    done_bases, t_used, n_done = 0, 0.0, 0
    chunk = max(threads * 4, 16)
    pos = 0
    while t_used < seconds and pos < r.n:
        idx = order[pos:pos + chunk]
        pos += len(idx)
        sub = r.subset(idx)
        t0 = time.perf_counter()
        O.dp_batch(g, sub.seq, sub.off, sub.v_start, sub.n_edits, n_threads=threads)
        t_used += time.perf_counter() - t0
        done_bases += int(sub.off[-1])
        n_done += len(idx)
    return done_bases / t_used, n_done, done_bases, t_used


def cpu_baseline(g, r, seconds: float = 15.0, seed: int = 11):
    """The oracle (Eq. 1, value-capped at the read's injected edits, OpenMP
    over reads) on a bounded seeded sample of the same reads, with every
    host thread, and on one thread on a shorter sample."""
    import oracle as O
    rng = np.random.default_rng(seed)
    order = rng.permutation(r.n)
    threads = O.num_threads()
    rate, n_done, done_bases, t_used = _oracle_rate(g, r, order, threads, seconds)
    rate1, n1, b1, t1 = _oracle_rate(g, r, order, 1, max(2.0, seconds / 3))
    return {"value": rate, "unit": "bases/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_done} of {r.n} reads (seeded), {done_bases} bases, {t_used:.1f} s, Eq.1 DP capped at "
                      f"the injected edit count, OpenMP over reads",
            "cpu": cpu_model(), "logical_cpus": os.cpu_count(),
            "one_thread": {"value": rate1, "unit": "bases/s", "sample": f"{n1} reads, {b1} bases, {t1:.1f} s"}}


def recorded_traffic(workload: str, lanes: int):
    """HBM traffic per launch of k_align from the committed rocprofv3 summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy calibration), only while
    the kernel source is the one that was profiled; else None."""
    import glob
    import hashlib
    import re
    root = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(root, "paper_2206_13574_amd", "csrc", "gwfa_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for f in sorted(glob.glob(os.path.join(root, "profiles", "k_align_*.md"))):
        m = re.search(r"```json\n(.*?)\n```", open(f).read(), re.S)
        if not m:
            continue
        d = json.loads(m.group(1))
        if d.get("workload") == workload and d.get("kernel_src_sha256_16") == sha and d.get("lanes") == lanes:
            return d["traffic_bytes_per_launch"], os.path.relpath(f, root)
    return None, None


def compare_mode(ctx, graph, batch, out, n, bases, res_exact, stream, ev, o, params):
    """One warm and one timed alignment launch of the resident (packed)
    batch in another mode; its distances against the exact ones."""
    import torch
    from paper_2206_13574_amd import gwfa
    gwfa.align_dev(ctx, graph, batch, out, o)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record(stream)
    gwfa.align_dev(ctx, graph, batch, out, o)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    res, _, _ = gwfa.fetch(out, n)
    ok = (res["status"] == 0) & (res_exact["status"] == 0)
    exc = (res["dist"] - res_exact["dist"])[ok].astype(np.int64)
    # a pruned read without a distance counts as over the exact distance
    n_over = int((exc > 0).sum()) + int((~ok).sum())
    return dict(params, align_ms=ms, bases_per_s=bases / (ms / 1000.0),
                frac_reads_over=n_over / n if n else 0.0,
                mean_excess=float(exc.mean()) if len(exc) else 0.0,
                min_excess=int(exc.min()) if len(exc) else 0, not_ok=int((~ok).sum()))


def measure(args, workload, steps, warmup, prune, compare, end_to_end=False):
    """Times `steps` steps of the whole path on one workload (after `warmup`
    untimed ones) and returns the fields of the benchmark line."""
    import torch
    from paper_2206_13574_amd import gwfa, tune

    t0 = time.time()
    g, r = make_workload(workload, args.reads)
    print(f"[bench] workload {workload}: {r.n} reads, {int(r.off[-1])} bases, graph {g.n_vtx} V "
          f"{g.n_edge} E ({time.time() - t0:.1f} s to generate)", file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)          # default priority
    ctx = gwfa.Context(0, stream=stream)
    cfg = tune.best_config(workload)
    if args.lanes:
        cfg["lanes"] = args.lanes
    if args.groups is not None:
        cfg["groups"] = args.groups
    ctx.config(**cfg)
    graph = gwfa.Graph.of(ctx, g)
    o = gwfa.opts(prune=prune, a_diff=args.a_diff, traceback=not args.no_traceback)
    with torch.cuda.stream(stream):
        batch = gwfa.upload_reads(ctx, r.seq, r.off, r.v_start)
        out = gwfa.alloc_out(ctx, r.n, (int(r.off[-1]) // 4 + 64 * r.n) if o.traceback else 0)
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)
    # the alignment of the resident batch is captured once as a HIP graph
    # (queue reset, screen pass, persistent alignment kernel) and replayed
    plan = gwfa.Plan(ctx, graph, batch, out, o)
    for i in range(warmup):
        tw = time.perf_counter()
        gwfa.pack_dev(ctx, batch, out.err)
        plan.launch()
        plan.finish()
        print(f"[bench] {workload} warm-up {i + 1}/{warmup}: {time.perf_counter() - tw:.2f} s", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    ctx.stats(reset=True)

    pack_ms, align_ms = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(steps):
        e0, e1, e2 = ev(), ev(), ev()
        e0.record(stream)
        gwfa.pack_dev(ctx, batch, out.err)
        e1.record(stream)
        plan.launch()
        plan.finish()   # re-runs of overflowed queries, if any (synchronises)
        e2.record(stream)
        pack_ms.append((e0, e1))
        align_ms.append((e1, e2))
        print(f"[bench] {workload} step {i + 1}/{steps} done at {time.perf_counter() - t_start:.2f} s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    pack_ms = [a.elapsed_time(b) for a, b in pack_ms]
    align_ms = [a.elapsed_time(b) for a, b in align_ms]
    st = ctx.stats()
    res, _, used = gwfa.fetch(out, r.n)
    bad = int((res["status"] != 0).sum())
    if bad:
        print(f"[bench] WARNING: {bad} reads without status OK", file=sys.stderr)
    if int(out.err.cpu().item()) != 0:
        print("[bench] WARNING: alphabet error flag set", file=sys.stderr)

    bases = int(r.off[-1])
    entries = st["entries"] / steps
    chunks = max(st["chunks"] / steps, entries)
    cross = st["crossings"] / steps
    admitted = st["admitted"] / steps
    b_entry = B_ENTRY + (B_ENTRY_TB if o.traceback else 0)
    b_cross = B_CROSS + (B_PUSH if o.traceback else 0)
    alg_bytes = entries * b_entry + chunks * B_CHUNK + cross * b_cross
    align_avg_s = float(np.mean(align_ms)) / 1000.0
    achieved = alg_bytes / align_avg_s / 1e9
    traffic, traffic_src = recorded_traffic(workload, cfg["lanes"])
    # phases of the kernel (thread-0 wall-clock ticks summed over workgroups):
    # the expansion with the extension of what it admits (entries, records,
    # their compare chunks) and the crossing rounds (crossings and the
    # extension of the crossed entries); chunks are split between the two in
    # proportion to the entries each extends (an approximation: the kernel
    # counts them together)
    ticks = [st["ticks_expand"], st["ticks_rounds"], st["ticks_merge"], st["ticks_prune"]]
    tsum = float(sum(ticks)) or 1.0
    share_x = admitted / (admitted + cross) if admitted + cross else 1.0
    phases = {}
    for name, ti, nbytes in (("expand", 0, entries * b_entry + chunks * share_x * B_CHUNK),
                             ("crossing_rounds", 1, cross * b_cross + chunks * (1 - share_x) * B_CHUNK),
                             ("merge", 2, 0.0)):
        sec = align_avg_s * ticks[ti] / tsum
        phases[name] = {"time_frac": ticks[ti] / tsum, "model_bytes": nbytes,
                        "GB/s": nbytes / sec / 1e9 if sec > 0 and nbytes else None,
                        "frac": nbytes / sec / 1e9 / HBM_PEAK_GBS if sec > 0 and nbytes else None}
    pack_avg_s = float(np.mean(pack_ms)) / 1000.0
    # context for the pack's rate: a plain device copy that moves the same
    # number of bytes (half read, half written), timed the same way
    with torch.cuda.stream(stream):
        half = int(bases * 1.25) // 2
        src_t = torch.empty(half, dtype=torch.uint8, device=dev)
        dst_t = torch.empty(half, dtype=torch.uint8, device=dev)
        cms = []
        for _ in range(4):
            c0, c1 = ev(), ev()
            c0.record(stream)
            dst_t.copy_(src_t)
            c1.record(stream)
            torch.cuda.synchronize()
            cms.append(c0.elapsed_time(c1))
        copy_gbs = 2 * half / (float(np.median(cms[1:])) / 1000.0) / 1e9
        del src_t, dst_t
    pack_bytes = bases * 1.25
    m = {
        "value": bases * steps / wall,
        "ms_per_step": wall * 1000.0 / steps,
        "config": {"workload": f"{workload}: {WORKLOADS[workload]}", "reads": r.n, "bases": bases,
                   "graph_vertices": g.n_vtx, "graph_edges": g.n_edge,
                   "mode": ["exact", "heuristic-prune", "learned-prune"][prune],
                   "a_diff": args.a_diff if prune == 1 else None, "traceback": bool(o.traceback),
                   "lanes_per_read": cfg["lanes"], "groups": cfg.get("groups", 0),
                   "dir_log2_max": cfg["dir_log2_max"], "dir_factor": cfg["dir_factor"],
                   "list_cap": cfg["list_cap"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": traffic_src,
                     "kernel": "k_align (persistent, one workgroup per read)",
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": align_avg_s * 1000.0,
                     "entries_per_launch": entries, "chunks_per_launch": chunks,
                     "crossings_per_launch": cross, "phases": phases},
        "pack": {"avg_ms": pack_avg_s * 1000.0, "GB/s": pack_bytes / pack_avg_s / 1e9,
                 "frac": pack_bytes / pack_avg_s / 1e9 / HBM_PEAK_GBS,
                 "same_traffic_copy_GB/s": copy_gbs,
                 "frac_of_copy": pack_bytes / pack_avg_s / 1e9 / copy_gbs},
        "reruns": st["reruns"] / steps,
        "not_ok": bad,
    }
    if compare and prune == 0:
        try:
            # the metric's comparison: learned pruning (and Algorithm 4) on the same
            # resident batch, outside the timed steps, against the exact distances
            from paper_2206_13574_amd import calibrate_prune, train_prune
            W = train_prune.load()
            ctx.mlp_load(W["w_bf16"], W["scale"])
            # the keep threshold calibrated on held-out sets of this workload's
            # shape when there is one, else the training-shape threshold
            shaped = calibrate_prune.load().get(workload)
            tau = float(shaped["tau"]) if shaped else W["tau"]
            tau_src = (f"held-out {workload}-shaped sets ({shaped['reads']} reads, graph seeds "
                       f"{shaped['graph_seeds']})" if shaped else "held-out training-shaped sets")
            # each mode at its own measured lanes per query (pruned wavefronts are
            # small: narrower workgroups keep more queries in flight)
            lanes_l = tune.best_lanes(workload, "learned")
            lanes_h = tune.best_lanes(workload, "heuristic")
            ctx.config(**dict(cfg, lanes=lanes_l))
            learned = compare_mode(ctx, graph, batch, out, r.n, bases, res, stream, ev,
                                   gwfa.opts(prune=gwfa.PRUNE_LEARNED, keep_threshold=tau, mlp_gate=W["gate"],
                                             mlp_period=W["period"], traceback=bool(o.traceback)),
                                   dict(tau=tau, tau_calibrated_on=tau_src, gate=W["gate"], period=W["period"],
                                        lanes=lanes_l))
            ctx.config(**dict(cfg, lanes=lanes_h))
            heuristic = compare_mode(ctx, graph, batch, out, r.n, bases, res, stream, ev,
                                     gwfa.opts(prune=gwfa.PRUNE_HEURISTIC, a_diff=50, traceback=bool(o.traceback)),
                                     dict(a_diff=50, lanes=lanes_h))
            m["compare"] = {"learned-prune": learned, "heuristic-prune": heuristic,
                            "exact_align_ms": align_avg_s * 1000.0, "exact_lanes": cfg["lanes"]}
        except Exception as e:   # the comparison must not cost the benchmark line
            print(f"[bench] comparison legs failed: {e}", file=sys.stderr, flush=True)
            m["compare"] = {"error": str(e)}
    if end_to_end and prune == 0:
        try:
            # the same batch from host memory through the host-buffer entry
            # point (validation, query sort, copies in, alignment, results and
            # walks back): a separate figure, never the line's value
            ctx.config(**cfg)
            cap = (bases // 4 + 64 * r.n) if o.traceback else 0
            torch.cuda.synchronize()
            th = time.perf_counter()
            code, res_h, _, _ = gwfa.align_host(ctx, graph, r.seq, r.off, r.v_start, o, path_cap=cap)
            e2e_s = time.perf_counter() - th
            same = bool(code == 0 and (res_h["dist"] == res["dist"]).all())
            m["end_to_end"] = {"entry": "gwfa_align_batch (host buffers, pageable)", "ms": e2e_s * 1000.0,
                               "bases/s": bases / e2e_s, "code": int(code), "same_distances": same}
            print(f"[bench] {workload} end to end from host buffers: {e2e_s:.2f} s", file=sys.stderr, flush=True)
        except Exception as e:   # this figure must not cost the benchmark line
            print(f"[bench] end-to-end leg failed: {e}", file=sys.stderr, flush=True)
            m["end_to_end"] = {"error": str(e)}
    plan.close()
    graph.close()
    ctx.close()
    return m, g, r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg4", choices=sorted(WORKLOADS))
    ap.add_argument("--secondary", default="cfg2", choices=sorted(WORKLOADS) + ["none"],
                    help="a second workload measured after the first (at most 5 steps), reported beside it")
    ap.add_argument("--reads", type=int, default=None)
    ap.add_argument("--lanes", type=int, default=None)
    ap.add_argument("--groups", type=int, default=None)
    ap.add_argument("--prune", type=int, default=0)
    ap.add_argument("--a-diff", type=int, default=0)
    ap.add_argument("--no-traceback", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the learned / heuristic pruning comparison after the timed steps")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-end-to-end", dest="end_to_end", action="store_false",
                    help="skip the one call through the host-buffer entry point after the timed steps")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling rocprof FETCH/WRITE counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (each query batch shards across GPUs by reads with "
              "no exchange; see the design notes) -- run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    m, g, r = measure(args, args.workload, args.steps, args.warmup, args.prune, not args.no_compare,
                      args.end_to_end)
    line = {
        "metric": "query bases aligned/s on 1 GPU; exact vs learned-prune at <=1% reads over ED",
        "value": m["value"],
        "unit": "bases/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
    }
    line.update({k: v for k, v in m.items() if k not in ("value", "ms_per_step")})
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host cores", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(g, r, seconds=args.cpu_seconds)
    del g, r
    if args.secondary != "none" and args.secondary != args.workload:
        try:
            s, _, _ = measure(args, args.secondary, min(args.steps, 5), 1, args.prune, False)
            line["secondary"] = {"value": s["value"], "unit": "bases/s", "ms_per_step": s["ms_per_step"],
                                 "steps": min(args.steps, 5), "config": s["config"],
                                 "roofline": {k: s["roofline"][k] for k in ("achieved", "frac", "avg_launch_ms",
                                                                              "alg_bytes_per_launch")},
                                 "not_ok": s["not_ok"]}
        except Exception as e:   # the secondary workload must not cost the benchmark line
            print(f"[bench] secondary workload failed: {e}", file=sys.stderr, flush=True)
            line["secondary"] = {"error": str(e)}
    if args.copy_calib:
        dev = torch.device("cuda", 0)
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device=dev)
        b = torch.empty(n, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        line["copy_calib_bytes"] = n
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
