"""Launch-shape autotuner: lanes per query and persistent workgroups.

`autotune` times the whole batch step for each candidate on a stratified
sample of the queries (every k-th query of the length-sorted batch, so long
and short queries are both represented) and keeps the fastest; the result is
cached per (device name, workload) in tune_cache.json beside this file.
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
    try:
        import torch
        return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    except Exception:
        return "cpu"


def best_config(workload: str) -> dict:
    c = _load().get(f"{_device_name()}|{workload}")
    out = dict(DEFAULT)
    if c:
        out.update({k: c[k] for k in DEFAULT if k in c})
    return out


def autotune(workload: str, g, r, sample: int = 4000, lanes=(64, 128, 256), groups=(0, 2048, 4096),
             repeats: int = 2, save: bool = True, log=print) -> dict:
    from . import gwfa
    import torch
    lens = r.off[1:] - r.off[:-1]
    order = np.argsort(-lens, kind="stable")
    k = max(1, r.n // sample)
    sub = r.subset(order[::k][:sample])
    best, best_t = None, float("inf")
    stream = torch.cuda.Stream()
    for ln in lanes:
        for gr in groups:
            cfg = dict(DEFAULT, lanes=ln, groups=gr)
            ctx = gwfa.Context(0, stream=stream)
            ctx.config(**cfg)
            graph = gwfa.Graph.of(ctx, g)
            with torch.cuda.stream(stream):
                batch = gwfa.upload_reads(ctx, sub.seq, sub.off, sub.v_start)
                out = gwfa.alloc_out(ctx, sub.n, int(sub.off[-1]) // 4 + 64 * sub.n)
            gwfa.step_dev(ctx, graph, batch, out, gwfa.opts())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(repeats):
                gwfa.step_dev(ctx, graph, batch, out, gwfa.opts())
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / repeats
            log(f"[tune] lanes={ln} groups={gr}: {t * 1000:.1f} ms")
            if t < best_t:
                best, best_t = cfg, t
            graph.close()
            ctx.close()
    if save:
        c = _load()
        c[f"{_device_name()}|{workload}"] = dict(best, ms=best_t * 1000.0, sample=sub.n)
        with open(_CACHE, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
    return best
