"""Autotuner of the launch shape and the arena tiles: lanes per query,
persistent workgroups, wavefront-list capacity and record-directory size and
growth of the first working-memory tier.

`autotune` times the whole batch step for each candidate on a stratified
sample of the queries (every k-th query of the length-sorted batch, so long
and short queries are both represented), searching one parameter at a time,
and keeps the fastest; the result is cached per (device, workload) in
tune_cache.json beside this file, which `best_config` reads.  With --mode
heuristic or learned it times that pruning mode (Algorithm 4 at a_diff 50,
or the trained network) at every lanes-per-query width on the workload's
exact configuration and caches the fastest as lanes_<mode> (`best_lanes`).
Usage: python -m paper_2206_13574_amd.tune --workload cfg2 [--mode learned]
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")

DEFAULT = dict(lanes=256, groups=0, dir_log2_max=16, list_cap=1 << 15, dir_factor=16)


def _load():
    try:
        with open(_CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _device_name():
    """Cache key of the device: its ISA and compute-unit count (the marketing
    name depends on which lookup tables the process found)."""
    try:
        import torch
        if not torch.cuda.is_available():
            return "cpu"
        p = torch.cuda.get_device_properties(0)
        return f"{p.gcnArchName.split(':')[0]}x{p.multi_processor_count}"
    except Exception:
        return "cpu"


def best_config(workload: str) -> dict:
    c = _load().get(f"{_device_name()}|{workload}")
    out = dict(DEFAULT)
    if c:
        out.update({k: c[k] for k in DEFAULT if k in c})
    return out


def best_lanes(workload: str, mode: str) -> int:
    """Lanes per query for a pruning mode ("heuristic" or "learned"): pruned
    wavefronts are small, so these modes may prefer narrower workgroups than
    the exact configuration; the exact configuration's lanes when none was
    measured."""
    c = _load().get(f"{_device_name()}|{workload}") or {}
    return int(c.get(f"lanes_{mode}", best_config(workload)["lanes"]))


def _mode_opts(mode: str):
    """Options and network weights (or None) of a mode."""
    from . import gwfa
    if mode == "exact":
        return gwfa.opts(), None
    if mode == "heuristic":
        return gwfa.opts(prune=gwfa.PRUNE_HEURISTIC, a_diff=50), None
    from . import train_prune
    W = train_prune.load()
    return gwfa.opts(prune=gwfa.PRUNE_LEARNED, keep_threshold=W["tau"], mlp_gate=W["gate"],
                     mlp_period=W["period"]), W


def _time_config(g, sub, cfg, repeats, stream, mode: str = "exact"):
    from . import gwfa
    import torch
    o, W = _mode_opts(mode)
    ctx = gwfa.Context(0, stream=stream)
    try:
        ctx.config(**cfg)
        if W is not None:
            ctx.mlp_load(W["w_bf16"], W["scale"])
        graph = gwfa.Graph.of(ctx, g)
        with torch.cuda.stream(stream):
            batch = gwfa.upload_reads(ctx, sub.seq, sub.off, sub.v_start)
            out = gwfa.alloc_out(ctx, sub.n, int(sub.off[-1]) // 4 + 64 * sub.n)
        gwfa.step_dev(ctx, graph, batch, out, o)     # warm-up (allocates the arenas)
        torch.cuda.synchronize()
        ctx.stats(reset=True)
        t0 = time.perf_counter()
        for _ in range(repeats):
            gwfa.step_dev(ctx, graph, batch, out, o)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / repeats
        reruns = ctx.stats()["reruns"]
        graph.close()
    finally:
        ctx.close()
    return t, reruns


# candidate values per parameter, searched one parameter at a time
# (a first-tier arena is about 2^dir_log2_max x 570 bytes per workgroup; the
# library caps each tier's workgroups by its share of the free device memory)
SPACE = dict(lanes=(128, 256, 512), groups=(512, 768, 0), list_cap=(1 << 13, 1 << 15, 1 << 16, 1 << 17),
             dir_factor=(16, 64, 256), dir_log2_max=(15, 16, 17, 18))


def autotune(workload: str, g, r, sample: int = 0, repeats: int = 2, save: bool = True, rounds: int = 2,
             space: dict = None, log=print) -> dict:
    """Coordinate search over lanes per query, persistent workgroups and the
    arena tiles (list capacity, directory size and growth) on a stratified
    sample of the batch (sample = 0: the whole batch, which is what to tune
    on: a sample too small to fill the GPU favours more lanes per query than
    the full batch does); every candidate's results must be complete (an
    overflow re-run counts against it through its time)."""
    import torch
    space = space or SPACE
    lens = r.off[1:] - r.off[:-1]
    order = np.argsort(-lens, kind="stable")
    if sample <= 0 or sample >= r.n:
        sub = r
    else:
        k = max(1, r.n // sample)
        sub = r.subset(order[::k][:sample])
    stream = torch.cuda.Stream()
    best = dict(DEFAULT)
    best_t, _ = _time_config(g, sub, best, repeats, stream)
    log(f"[tune] start {best}: {best_t * 1000:.1f} ms")
    seen = {tuple(sorted(best.items())): best_t}
    for rd in range(rounds):
        changed = False
        for key, values in space.items():
            for v in values:
                cfg = dict(best, **{key: v})
                sig = tuple(sorted(cfg.items()))
                if sig in seen:
                    continue
                t, reruns = _time_config(g, sub, cfg, repeats, stream)
                seen[sig] = t
                log(f"[tune] {key}={v}: {t * 1000:.1f} ms (re-runs {reruns})")
                if t < best_t * 0.98:
                    best, best_t, changed = cfg, t, True
        if not changed:
            break
    log(f"[tune] best {best}: {best_t * 1000:.1f} ms")
    if save:
        c = _load()
        key = f"{_device_name()}|{workload}"
        c[key] = dict(c.get(key, {}), **best, ms=best_t * 1000.0, sample=sub.n)
        with open(_CACHE, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
    return best


def tune_mode_lanes(workload: str, g, r, mode: str, repeats: int = 2, save: bool = True, log=print) -> int:
    """Lanes per query for a pruning mode on the whole batch, the other
    parameters at the workload's exact configuration."""
    import torch
    stream = torch.cuda.Stream()
    base = best_config(workload)
    times = {}
    for lanes in (64, 128, 256, 512):
        t, reruns = _time_config(g, r, dict(base, lanes=lanes), repeats, stream, mode)
        times[lanes] = t
        log(f"[tune] {mode} lanes={lanes}: {t * 1000:.1f} ms (re-runs {reruns})")
    best = min(times, key=times.get)
    log(f"[tune] {mode}: best lanes {best}")
    if save:
        c = _load()
        key = f"{_device_name()}|{workload}"
        c[key] = dict(c.get(key, {}), **{f"lanes_{mode}": best, f"ms_{mode}": times[best] * 1000.0})
        with open(_CACHE, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
    return best


def main(argv=None):
    import argparse
    from . import synth
    ap = argparse.ArgumentParser(description="autotune the launch shape and arena tiles for a workload")
    ap.add_argument("--workload", default="cfg2", choices=("cfg1", "cfg2", "cfg3", "cfg4", "cfg4b"))
    ap.add_argument("--sample", type=int, default=0, help="queries to time (0: all)")
    ap.add_argument("--repeats", type=int, default=2)
    ap.add_argument("--mode", default="exact", choices=("exact", "heuristic", "learned"),
                    help="exact: the full search; a pruning mode: its lanes per query only")
    a = ap.parse_args(argv)
    g, r = synth.cfg4(sparse=True) if a.workload == "cfg4b" else getattr(synth, a.workload)()
    if a.mode == "exact":
        autotune(a.workload, g, r, sample=a.sample, repeats=a.repeats, log=lambda m: print(m, flush=True))
    else:
        tune_mode_lanes(a.workload, g, r, a.mode, repeats=a.repeats, log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    main()
