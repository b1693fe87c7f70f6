"""GPU parity of the host-buffer entry points (gwfa_align for one query,
gwfa_align_batch), valid inputs only: distance and end bit-exact against
the dense oracle, walks re-scored, and a path buffer that is too small."""
import numpy as np
import pytest

import oracle as O
from paper_2206_13574_amd import synth
from tests.test_gpu_parity import reads_of

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-host] {msg}", flush=True)


def test_host_entry_points_on_cfg1(gpu_lib):
    gw = gpu_lib
    g, r = synth.cfg1()
    ctx = gw.Context(0)
    graph = gw.Graph.of(ctx, g)
    try:
        say("gwfa_align, one query at a time")
        for i in range(0, r.n, 5):
            q = r.read(i)
            code, res, walk = gw.align_one(ctx, graph, q, int(r.v_start[i]))
            d, ev, ej, _ = O.dp_dense(g, q, int(r.v_start[i]))
            assert code == gw.OK and (res["status"], res["dist"], res["end_v"], res["end_off"]) == (0, d, ev, ej), i
            assert walk[0] == r.v_start[i] and O.is_walk(g, walk)
            assert O.ed_global(q, O.spell_walk(g, walk, ej)) == d
        say("gwfa_align_batch")
        sub = r.subset(np.arange(20))
        code, res, path, need = gw.align_host(ctx, graph, sub.seq, sub.off, sub.v_start, gw.opts(),
                                              path_cap=int(sub.off[-1]) + 64 * sub.n)
        assert code == gw.OK
        for i in range(sub.n):
            d, ev, ej, _ = O.dp_dense(g, sub.read(i), int(sub.v_start[i]))
            assert (res[i]["dist"], res[i]["end_v"], res[i]["end_off"]) == (d, ev, ej), i
            walk = path[res[i]["path_off"]:res[i]["path_off"] + res[i]["path_len"]]
            assert O.ed_global(sub.read(i), O.spell_walk(g, walk, ej)) == d
        say("gwfa_align_batch, path buffer too small")
        code2, res2, _, need2 = gw.align_host(ctx, graph, sub.seq, sub.off, sub.v_start, gw.opts(), path_cap=3)
        assert code2 == gw.ERR_PATH_CAP and need2 == need
        assert (res2["dist"] == res["dist"]).all()
    finally:
        graph.close()
        ctx.close()
