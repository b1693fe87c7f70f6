"""GPU parity of the free end gap in the query (opts.query_end_free = e: up
to e trailing query bases left unaligned at no cost, the best over rows
|q| - e .. |q|, ties to the longest aligned prefix): distance, end, clip and
work bit-exact against the dense oracle and the Algorithms 1-4 transcription
in both forms, walks re-scored on the aligned prefix, CIGARs ending in the
soft clip."""
import numpy as np
import pytest

import oracle as O
from paper_2206_13574_amd import synth
from tests import refs
from tests.test_gpu_parity import union_graph, reads_of

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-clip] {msg}", flush=True)


@pytest.fixture(scope="module")
def G(gpu_lib):
    ctx = gpu_lib.Context(0)
    yield gpu_lib, ctx
    ctx.close()


def _check_cigar(q, T, ops, d, clip):
    assert refs.cigar_cost(q, T, ops) == d
    if clip > 0:
        assert (int(ops[-1]) & 15) == 4 and int(ops[-1]) >> 4 == clip
    else:
        assert all((int(w) & 15) != 4 for w in ops)


@pytest.mark.parametrize("e", [1, 4, 1000])
def test_clip_tiny_random_graphs_both_forms(G, e):
    gw, ctx = G
    rng = np.random.default_rng(5600 + e)
    cases = []
    for _ in range(1500):
        labels, edges, q, vs = refs.random_case(rng, n_vtx=int(rng.integers(1, 7)),
                                                max_label=40 if rng.random() < 0.2 else 6, p_edge=0.35,
                                                qlen=int(rng.integers(0, 30)))
        L = len(labels[vs])
        j0 = int(rng.integers(0, L + 1)) if rng.random() < 0.5 else 0
        j1 = int(rng.integers(j0, L + 1)) if rng.random() < 0.5 else j0
        cases.append((labels, edges, q, vs, j0, j1, int(rng.integers(0, len(labels)))))
    g, base = union_graph([c[:4] for c in cases])
    graph = gw.Graph.of(ctx, g)
    o = gw.opts(query_end_free=e)
    try:
        seq, off = reads_of([c[2] for c in cases])
        n = len(cases)
        vs_all = np.array([c[3] + b for c, b in zip(cases, base)], np.int32)
        dev = lambda x: ctx.torch.from_numpy(np.ascontiguousarray(x, np.int32)).to(ctx.tdev)
        j0s = np.array([c[4] for c in cases], np.int32)
        j1s = np.array([c[5] for c in cases], np.int32)
        ves = np.array([c[6] + b for c, b in zip(cases, base)], np.int32)
        out = {}
        for form, ve in (("extension", None), ("global", ves)):
            say(f"e = {e}, {form} form, {n} tiny graphs, one launch, then CIGARs")
            batch = gw.upload_reads(ctx, seq, off, vs_all)
            buf = gw.alloc_out(ctx, n, int(off[-1]) * 4 + 256 * n)
            gw.step_dev(ctx, graph, batch, buf, o, None if ve is None else dev(ve), dev(j0s), dev(j1s))
            res, path, _ = gw.fetch(buf, n)
            out[form] = (res, path, gw.cigar_dev(ctx, graph, batch, buf))
    finally:
        graph.close()
    n_clip = 0
    for form in ("extension", "global"):
        res, path, (ops, coff, clen) = out[form]
        for i, (labels, edges, q, vs, j0, j1, ve) in enumerate(cases):
            vee = ve if form == "global" else -1
            ee = min(e, len(q))
            d, ev, ej, clip = O.dp_dense_clip((labels, edges), q, vs, ee, j0=j0, j1=j1, v_e=vee)
            r = res[i]
            if d < 0:
                assert r["status"] == gw.ST_UNREACHABLE, (form, i)
                continue
            wf = O.gwf((labels, edges), q, vs, j0=j0, j1=j1, v_e=vee, e=ee)
            assert (r["status"], r["dist"], r["end_v"] - base[i], r["end_off"], r["clip"], r["work"]) == \
                (0, d, ev, ej, clip, wf["work"]), (form, i, labels, edges, q, vs, j0, j1, ve)
            assert wf["clip"] == clip
            n_clip += clip > 0
            so = int(r["start_off"])
            p = path[r["path_off"]:r["path_off"] + r["path_len"]]
            assert j0 <= so <= j1 and p[0] == vs + base[i] and O.is_walk(g, p)
            T = O.spell_walk(g, p, ej)[so:]
            assert O.ed_global(q[:len(q) - clip], T) == d
            assert clen[i] >= 0
            _check_cigar(q, T, ops[coff[i]:coff[i] + clen[i]], d, clip)
    assert n_clip > 0


def test_clip_zero_is_the_default(G):
    """query_end_free = 0 gives the same results, field by field, as the
    default options."""
    gw, ctx = G
    g, r = synth.cfg1()
    qs = [r.read(i) for i in range(r.n)]
    graph = gw.Graph.of(ctx, g)
    try:
        seq, off = reads_of(qs)
        say("cfg1, query_end_free 0 against the defaults")
        a, pa = gw.align(ctx, graph, seq, off, np.asarray(r.v_start, np.int32))
        b, pb = gw.align(ctx, graph, seq, off, np.asarray(r.v_start, np.int32), gw.opts(query_end_free=0))
    finally:
        graph.close()
    for f in ("status", "dist", "end_v", "end_off", "work", "clip", "start_off"):
        assert np.array_equal(a[f], b[f]), f
    assert all(np.array_equal(x, y) for x, y in zip(pa, pb))
    assert not a["clip"].any()


def test_clip_cfg1_reads_with_adapter_tails(G):
    """Reads of the small workload with random tails appended (bases that
    are not in the graph): with e at least the tail length the tail is
    clipped, exact and under Algorithm 4, and CIGARs re-score to the
    distance."""
    gw, ctx = G
    g, r = synth.cfg1()
    rng = np.random.default_rng(5610)
    qs = []
    for i in range(r.n):
        tail = bytes(b"ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(0, 40))))
        qs.append(r.read(i) + tail)
    e = 50
    graph = gw.Graph.of(ctx, g)
    try:
        seq, off = reads_of(qs)
        n = r.n
        say(f"cfg1 reads + tails, e = {e}: exact + CIGAR")
        batch = gw.upload_reads(ctx, seq, off, np.asarray(r.v_start, np.int32))
        buf = gw.alloc_out(ctx, n, int(off[-1]) * 2 + 256 * n)
        gw.step_dev(ctx, graph, batch, buf, gw.opts(query_end_free=e))
        res, path, _ = gw.fetch(buf, n)
        ops, coff, clen = gw.cigar_dev(ctx, graph, batch, buf)
        for i in range(n):
            d, ev, ej, clip = O.dp_dense_clip(g, qs[i], int(r.v_start[i]), min(e, len(qs[i])))
            ref = O.gwf(g, qs[i], int(r.v_start[i]), e=min(e, len(qs[i])))
            x = res[i]
            assert (x["status"], x["dist"], x["end_v"], x["end_off"], x["clip"], x["work"]) == \
                (0, d, ev, ej, clip, ref["work"]), i
            p = path[x["path_off"]:x["path_off"] + x["path_len"]]
            T = O.spell_walk(g, p, ej)
            _check_cigar(qs[i], T, ops[coff[i]:coff[i] + clen[i]], d, clip)
        assert (res["clip"] > 0).sum() > n // 2
        for a in (8, 30):
            say(f"cfg1 reads + tails, e = {e}, Algorithm 4 a_diff {a}")
            res2, _ = gw.align(ctx, graph, seq, off, np.asarray(r.v_start, np.int32),
                               gw.opts(prune=gw.PRUNE_HEURISTIC, a_diff=a, query_end_free=e))
            for i in range(n):
                ref = O.gwf(g, qs[i], int(r.v_start[i]), a_diff=a, e=min(e, len(qs[i])))
                assert (res2[i]["dist"], res2[i]["end_v"], res2[i]["end_off"], res2[i]["clip"], res2[i]["work"]) == \
                    (ref["dist"], ref["end_v"], ref["end_j"], ref["clip"], ref["work"]), (i, a)
    finally:
        graph.close()


def test_clip_negative_is_an_argument_error(G):
    """A negative query end gap, and a walk end flag other than 0 or 1, are
    argument errors; a query end gap above |q| acts as |q|."""
    gw, ctx = G
    g = synth.Graph.from_labels(["ACGT"], [])
    graph = gw.Graph.of(ctx, g)
    seq, off = np.frombuffer(b"ACG", np.uint8), np.array([0, 3], np.int64)
    try:
        with pytest.raises(gw.GwfaError) as ei:
            gw.align(ctx, graph, seq, off, np.zeros(1, np.int32), gw.opts(query_end_free=-1))
        assert ei.value.code == gw.ERR_ARG
        o = gw.opts()
        o.walk_end_free = 2
        with pytest.raises(gw.GwfaError) as ei:
            gw.align(ctx, graph, seq, off, np.zeros(1, np.int32), o)
        assert ei.value.code == gw.ERR_ARG
        a, _ = gw.align(ctx, graph, np.frombuffer(b"TTT", np.uint8), off, np.zeros(1, np.int32),
                        gw.opts(query_end_free=1000))
        assert (a[0]["status"], a[0]["dist"], a[0]["clip"]) == (0, 0, 3)
    finally:
        graph.close()
