"""The error and status contract of the C ABI, one concern per test.

Graph errors (Definition 2.1: non-empty labels over A, C, G, T, edges
between existing vertices), argument and option errors of the host-buffer
and device entry points (all returned before any kernel is launched), the
per-query status of `opts.max_score`, and the global form with one end
vertex shared by a batch (`opts.end_vertex`) against the dense oracle.
Queries whose start vertex, start window or end vertex is out of range get
a per-query status (GWFA_ST_BAD_INPUT from the screen pass) in
tests/test_gpu_parity.py, tests/test_gpu_start.py and
tests/test_gpu_global.py."""
import numpy as np
import pytest

import oracle as O
from paper_2206_13574_amd import synth
from tests import refs
from tests.test_gpu_parity import reads_of

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-errors] {msg}", flush=True)


@pytest.fixture(scope="module")
def G(gpu_lib):
    ctx = gpu_lib.Context(0)
    yield gpu_lib, ctx
    ctx.close()


def test_graph_create_errors(G):
    gw, ctx = G
    say("graph errors")
    cases = [
        ((b"ACGT", [0, 2, 2, 4], [0], [1]), gw.ERR_EMPTY_LABEL),
        ((b"ACGT", [0, 2, 4], [0], [3]), gw.ERR_VERTEX),
        ((b"ACGT", [0, 2, 4], [-1], [1]), gw.ERR_VERTEX),
        ((b"ACXT", [0, 2, 4], [0], [1]), gw.ERR_ALPHABET),
        ((b"ACNT", [0, 4], [], []), gw.ERR_ALPHABET),
        ((b"ACGT", [1, 2, 4], [0], [1]), gw.ERR_ARG),          # offsets must start at 0
        ((b"ACGT", [0, 3, 2], [0], [1]), gw.ERR_ARG),          # and never decrease
    ]
    for (seq, off, src, dst), code in cases:
        with pytest.raises(gw.GwfaError) as e:
            gw.Graph(ctx, seq, np.array(off, np.int64), src, dst)
        assert e.value.code == code, (seq, off, src, dst)
    # lower case, self-loops and repeated edges are accepted
    g = gw.Graph(ctx, b"acgtTT", np.array([0, 4, 6], np.int64), [0, 0, 1, 1], [1, 1, 1, 0])
    g.close()


def test_host_entry_argument_errors(G):
    """gwfa_align_batch validates everything on the host before any device
    work: alphabet, start vertices, options."""
    gw, ctx = G
    g = synth.Graph.from_labels(["ACGT", "TT"], [(0, 1)])
    graph = gw.Graph.of(ctx, g)
    try:
        say("host entry: alphabet, vertex and option errors")
        seq, off = reads_of([b"ACGTT", b"ACNT"])
        assert gw.align_host(ctx, graph, seq, off, [0, 0])[0] == gw.ERR_ALPHABET
        seq, off = reads_of([b"ACGTT"])
        assert gw.align_host(ctx, graph, seq, off, [5])[0] == gw.ERR_VERTEX
        assert gw.align_host(ctx, graph, seq, off, [-1])[0] == gw.ERR_VERTEX
        assert gw.align_host(ctx, graph, seq, off, [0], gw.opts(end_vertex=2))[0] == gw.ERR_VERTEX
        assert gw.align_host(ctx, graph, seq, off, [0], gw.opts(end_vertex=-2))[0] == gw.ERR_ARG
        assert gw.align_host(ctx, graph, seq, off, [0], gw.opts(prune=gw.PRUNE_HEURISTIC, a_diff=0))[0] == \
            gw.ERR_ARG
        assert gw.align_host(ctx, graph, seq, off, [0], gw.opts(prune=gw.PRUNE_LEARNED))[0] == gw.ERR_UNSUPPORTED
        assert gw.align_host(ctx, graph, seq, off, [0], gw.opts(prune=3))[0] == gw.ERR_ARG
        assert gw.align_host(ctx, graph, seq, off, [0], gw.opts(max_score=-2))[0] == gw.ERR_ARG
        assert gw.align_host(ctx, graph, seq, off, [0], gw.opts(query_end_free=-1))[0] == gw.ERR_ARG
        bad = gw.opts()
        bad.traceback = 2
        assert gw.align_host(ctx, graph, seq, off, [0], bad)[0] == gw.ERR_ARG
        bad = gw.opts()
        bad.walk_end_free = 3
        assert gw.align_host(ctx, graph, seq, off, [0], bad)[0] == gw.ERR_ARG
        # read offsets must start at 0 and never decrease
        assert gw.align_host(ctx, graph, seq, np.array([1, 5], np.int64), [0])[0] == gw.ERR_ARG
        assert gw.align_host(ctx, graph, b"ACGTTACG", np.array([0, 5, 3], np.int64), [0, 0])[0] == gw.ERR_ARG
    finally:
        graph.close()


def test_device_entry_argument_errors(G):
    """The device entry points check their options and the shared end vertex
    on the host and return before any launch."""
    gw, ctx = G
    g = synth.Graph.from_labels(["ACGT", "TT", "GA"], [(0, 1), (1, 2), (2, 1)])
    graph = gw.Graph.of(ctx, g)
    try:
        say("device entry: option errors")
        seq, off = reads_of([b"ACGT"])
        for o, code in [(gw.opts(end_vertex=3), gw.ERR_VERTEX), (gw.opts(end_vertex=-5), gw.ERR_ARG),
                        (gw.opts(prune=gw.PRUNE_HEURISTIC, a_diff=-1), gw.ERR_ARG),
                        (gw.opts(prune=gw.PRUNE_LEARNED), gw.ERR_UNSUPPORTED),
                        (gw.opts(query_end_free=-3), gw.ERR_ARG)]:
            with pytest.raises(gw.GwfaError) as e:
                gw.align(ctx, graph, seq, off, np.zeros(1, np.int32), o)
            assert e.value.code == code
        # a shared end vertex and per-query end vertices together
        with pytest.raises(gw.GwfaError) as e:
            gw.align(ctx, graph, seq, off, np.zeros(1, np.int32), gw.opts(end_vertex=1), v_end=np.ones(1, np.int32))
        assert e.value.code == gw.ERR_ARG
    finally:
        graph.close()


def test_max_score_is_a_per_query_status(G):
    """A query whose distance exceeds opts.max_score stops there with status
    GWFA_ST_MAX_SCORE; the others in the same launch are exact."""
    gw, ctx = G
    g, r = synth.cfg1()
    sub = r.subset(np.arange(12))
    qs = [sub.read(i) for i in range(sub.n)]
    dist = [O.dp_dense(g, q, int(sub.v_start[i]))[0] for i, q in enumerate(qs)]
    cap = int(np.median(dist))
    say(f"max_score {cap}, distances {dist}")
    graph = gw.Graph.of(ctx, g)
    try:
        for tb in (True, False):
            res, paths = gw.align(ctx, graph, sub.seq, sub.off, sub.v_start, gw.opts(max_score=cap, traceback=tb))
            for i in range(sub.n):
                if dist[i] <= cap:
                    assert (res[i]["status"], res[i]["dist"]) == (gw.ST_OK, dist[i]), i
                else:
                    assert (res[i]["status"], res[i]["dist"], res[i]["end_v"]) == (gw.ST_MAX_SCORE, -1, -1), i
                    assert res[i]["path_len"] == 0 and res[i]["path_off"] == -1
    finally:
        graph.close()


def test_shared_end_vertex_on_medium_graphs(G):
    """Global form with opts.end_vertex: one end vertex for every query of a
    launch, on medium graphs with cycles: distance bit-exact against the
    dense global oracle, unreachable end vertices reported, walks end at the
    end vertex and re-score over their whole string."""
    gw, ctx = G
    rng = np.random.default_rng(7301)
    n_reach = n_unreach = 0
    for case in range(6):
        labels, edges, _, _, _ = refs.medium_case(rng)
        g = synth.Graph.from_labels(labels, edges)
        ve = int(rng.integers(len(labels) // 2, len(labels)))
        qs, vs = [], []
        for _ in range(24):
            v0 = int(rng.integers(0, len(labels)))
            t, _ = refs.spell_random_walk(rng, labels, edges, v0, int(rng.integers(20, 400)))
            qs.append(refs.mutate(rng, t, float(rng.uniform(0, 0.1))))
            vs.append(v0)
        seq, off = reads_of(qs)
        say(f"medium graph {case}: {len(labels)} V, end vertex {ve}, {len(qs)} queries")
        graph = gw.Graph.of(ctx, g)
        try:
            res, paths = gw.align(ctx, graph, seq, off, np.array(vs, np.int32), gw.opts(end_vertex=ve),
                                  path_cap=int(off[-1]) * 8 + 4096 * len(qs))
        finally:
            graph.close()
        for i, q in enumerate(qs):
            d = O.dp_dense_global((labels, edges), q, vs[i], ve)
            if d < 0:
                assert res[i]["status"] == gw.ST_UNREACHABLE, (case, i)
                n_unreach += 1
                continue
            n_reach += 1
            assert (res[i]["status"], res[i]["dist"], res[i]["end_v"], res[i]["end_off"]) == \
                (0, d, ve, len(labels[ve])), (case, i)
            p = [int(x) for x in paths[i]]
            assert p[0] == vs[i] and p[-1] == ve and O.is_walk(g, p)
            assert O.ed_global(q, O.spell_walk(g, p, len(labels[ve]))) == d
    assert n_reach > 20
