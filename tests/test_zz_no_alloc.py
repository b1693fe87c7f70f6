"""The entry point that allocates nothing (gwfa_align_batch_static_dev, for
callers that cannot allocate device memory) against the existing device
entry point gwfa_align_batch_dev on the same inputs: status, distance, end,
work, scores, start offset and clip bit-exact, on calls in a row (later ones
with smaller batches), so later calls run on memory earlier ones used.  The
traced walk is one of possibly several optimal walks (which one depends on
the order in which crossings were claimed), so each returned walk is checked
instead: it starts at the start vertex, follows edges, ends at the end cell,
and its string is at the distance from the query."""
import numpy as np
import pytest

import oracle as O
from paper_2206_13574_amd import synth
from tests import refs
from tests.test_gpu_parity import union_graph, reads_of

pytestmark = pytest.mark.gpu

FIELDS = ("status", "dist", "end_v", "end_off", "work", "n_scores", "start_off", "clip")


def say(msg):
    print(f"[gpu-static] {msg}", flush=True)


def _run(gw, ctx, graph, seq, off, vs, o, static):
    n = len(off) - 1
    batch = gw.upload_reads(ctx, seq, off, vs)
    out = gw.alloc_out(ctx, n, int(off[-1]) * 2 + 256 * n)
    gw.pack_dev(ctx, batch, out.err)
    if static:
        gw.align_static_dev(ctx, graph, batch, out, o)
    else:
        gw.align_dev(ctx, graph, batch, out, o)
    ctx.torch.cuda.synchronize()
    res, path, _ = gw.fetch(out, n)
    walks = [tuple(path[r["path_off"]:r["path_off"] + r["path_len"]]) if r["path_off"] >= 0 else None for r in res]
    return res, walks


def _same(a, b):
    (ra, wa), (rb, wb) = a, b
    for f in FIELDS:
        assert (ra[f] == rb[f]).all(), f
    assert [w is None for w in wa] == [w is None for w in wb]


def _walks_valid(g, qs, vs, res, walks, exact=True):
    """Exact runs: the walk's string is at the distance from the query.
    Pruned runs: the walk is a witness, at most the reported distance."""
    for i, w in enumerate(walks):
        if w is None:
            continue
        w = [int(x) for x in w]
        assert w[0] == int(vs[i]) and w[-1] == int(res[i]["end_v"]) and O.is_walk(g, w), i
        e = O.ed_banded(qs[i], O.spell_walk(g, w, int(res[i]["end_off"])), int(res[i]["dist"]))
        assert (e == res[i]["dist"]) if exact else (0 <= e <= res[i]["dist"]), (i, e, int(res[i]["dist"]))


def test_static_entry_point_matches_the_device_entry_point(gpu_lib):
    gw = gpu_lib
    rng = np.random.default_rng(8801)
    cases = [refs.random_case(rng, n_vtx=int(rng.integers(1, 8)), max_label=int(rng.integers(1, 7)),
                              p_edge=float(rng.uniform(0.1, 0.5)), qlen=int(rng.integers(0, 40)))
             for _ in range(1500)]
    g, base = union_graph(cases)
    qs = [c[2] for c in cases]
    vs = np.array([c[3] + b for c, b in zip(cases, base)], np.int32)
    ctx = gw.Context(0)
    graph = gw.Graph.of(ctx, g)
    try:
        for n, o in ((1500, gw.opts()), (300, gw.opts()), (1500, gw.opts(prune=gw.PRUNE_HEURISTIC, a_diff=6)),
                     (700, gw.opts(traceback=False))):
            seq, off = reads_of(qs[:n])
            say(f"tiny graphs: {n} queries, prune={o.prune} traceback={o.traceback}")
            st = _run(gw, ctx, graph, seq, off, vs[:n], o, static=True)
            assert (st[0]["status"] == 0).all()
            _same(st, _run(gw, ctx, graph, seq, off, vs[:n], o, static=False))
            _walks_valid(g, qs[:n], vs[:n], *st, exact=o.prune == 0)
    finally:
        graph.close()
        ctx.close()


def test_static_entry_point_on_cfg1_reads_twice(gpu_lib):
    gw = gpu_lib
    g, r = synth.cfg1()
    ctx = gw.Context(0)
    graph = gw.Graph.of(ctx, g)
    try:
        for n in (50, 17):
            sub = r.subset(np.arange(n))
            say(f"cfg1: {n} reads")
            st = _run(gw, ctx, graph, sub.seq, sub.off, sub.v_start, gw.opts(), static=True)
            assert (st[0]["status"] == 0).all()
            _same(st, _run(gw, ctx, graph, sub.seq, sub.off, sub.v_start, gw.opts(), static=False))
            _walks_valid(g, [sub.read(i) for i in range(n)], sub.v_start, *st)
    finally:
        graph.close()
        ctx.close()


def test_static_entry_point_refuses_too_many_queries(gpu_lib):
    gw = gpu_lib
    ctx = gw.Context(0)
    g = synth.Graph.from_labels(["ACGT"], [])
    graph = gw.Graph.of(ctx, g)
    try:
        import ctypes
        code = gw._lib.gwfa_align_batch_static_dev(ctx.h, graph.h, (1 << 20) + 1, None, None, None, None,
                                                   ctypes.byref(gw.opts()), None, None, 0, None, None)
        assert code == gw.ERR_ARG
        assert b"at most" in gw._lib.gwfa_last_error(ctx.h)
    finally:
        graph.close()
        ctx.close()
