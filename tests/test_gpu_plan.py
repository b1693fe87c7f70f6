"""Captured launches (gwfa_plan_*): every replay of the HIP graph, with
eager library work between replays, equals the eager call; queries that
overflow the first tier are completed by gwfa_plan_finish."""
import numpy as np
import pytest

import oracle as O
from paper_2206_13574_amd import synth

pytestmark = pytest.mark.gpu

FIELDS = ["dist", "end_v", "end_off", "status", "path_len", "work"]


def say(msg):
    print(f"[gpu-plan] {msg}", flush=True)


@pytest.mark.parametrize("small", [False, True])
def test_plan_replays_equal_eager(gpu_lib, small):
    gw = gpu_lib
    ctx = gw.Context(0)
    if small:   # tiny first tier: many queries overflow and are re-run by finish()
        ctx.config(lanes=128, dir_log2_max=10, list_cap=1024, dir_factor=1)
    g, r = synth.cfg2(n_reads=150 if small else 400)
    graph = gw.Graph.of(ctx, g)
    batch = gw.upload_reads(ctx, r.seq, r.off, r.v_start)
    cap = int(r.off[-1]) // 4 + 64 * r.n
    o = gw.opts()
    eager = gw.alloc_out(ctx, r.n, cap)
    say(f"eager small={small}")
    gw.step_dev(ctx, graph, batch, eager, o)
    ctx.torch.cuda.synchronize()
    ref, _, _ = gw.fetch(eager, r.n)
    st = ctx.stats(reset=True)
    if small:
        assert st["reruns"] > 0
    outp = gw.alloc_out(ctx, r.n, cap)
    plan = gw.Plan(ctx, graph, batch, outp, o)
    other = gw.alloc_out(ctx, r.n, cap)
    for rep in range(3):
        say(f"replay {rep}")
        outp.res.zero_()
        plan.launch()
        plan.finish()
        got, path, used = gw.fetch(outp, r.n)
        for f in FIELDS:
            assert np.array_equal(got[f], ref[f]), (rep, f)
        for k in range(0, r.n, 97):
            p = path[got[k]["path_off"]:got[k]["path_off"] + got[k]["path_len"]]
            assert O.is_walk(g, p) and p[0] == r.v_start[k] and p[-1] == got[k]["end_v"]
        # eager work between replays, on the same context and stream
        gw.step_dev(ctx, graph, batch, other, gw.opts(prune=gw.PRUNE_HEURISTIC, a_diff=50))
        ctx.torch.cuda.synchronize()
    plan.close()
    graph.close()
    ctx.close()
