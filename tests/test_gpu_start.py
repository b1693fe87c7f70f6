"""GPU parity of walks that start inside the start vertex (gwfa_align_at_dev):
Eq. 1 with the initial cell (0, v_s, j0), in extension mode and in the
global form, against the dense oracle (distance, end) and the Algorithms
1-4 transcription (work counts), walks re-scored from offset j0, CIGARs
checked against the spelled walk, and out-of-range offsets rejected per
query."""
import numpy as np
import pytest

import oracle as O
from paper_2206_13574_amd import synth
from tests import refs
from tests.test_gpu_parity import union_graph, reads_of

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-start] {msg}", flush=True)


@pytest.fixture(scope="module")
def G(gpu_lib):
    ctx = gpu_lib.Context(0)
    yield gpu_lib, ctx
    ctx.close()


def _spell_from(g, path, j0, end_off):
    s = O.spell_walk(g, path, end_off)
    return s[j0:]


def _tiny_cases(seed, n):
    rng = np.random.default_rng(seed)
    cases = []
    for _ in range(n):
        labels, edges, q, vs = refs.random_case(rng, n_vtx=int(rng.integers(1, 7)), max_label=5, p_edge=0.35,
                                                qlen=int(rng.integers(0, 30)))
        cases.append((labels, edges, q, vs, int(rng.integers(0, len(labels[vs]) + 1)),
                      int(rng.integers(0, len(labels)))))
    return cases


def test_start_offset_extension_tiny_random_graphs(G):
    gw, ctx = G
    cases = _tiny_cases(5501, 2000)
    g, base = union_graph([c[:4] for c in cases])
    say(f"extension form, {len(cases)} tiny graphs with start offsets, one launch")
    graph = gw.Graph.of(ctx, g)
    try:
        seq, off = reads_of([c[2] for c in cases])
        res, paths = gw.align(ctx, graph, seq, off, np.array([c[3] + b for c, b in zip(cases, base)], np.int32),
                              start_off=np.array([c[4] for c in cases], np.int32),
                              path_cap=int(off[-1]) * 4 + 256 * len(cases))
    finally:
        graph.close()
    for i, (labels, edges, q, vs, j0, _) in enumerate(cases):
        d, ev, ej = O.dp_dense_at((labels, edges), q, vs, j0)
        wf = O.gwf((labels, edges), q, vs, j0=j0)
        r = res[i]
        assert (r["status"], r["dist"], r["end_v"] - base[i], r["end_off"], r["work"], r["start_off"]) == \
            (0, d, ev, ej, wf["work"], j0), (i, labels, edges, q, vs, j0)
        p = paths[i]
        assert p[0] == vs + base[i] and p[-1] == ev + base[i] and O.is_walk(g, p)
        assert O.ed_global(q, _spell_from(g, p, j0, ej)) == d


def test_start_offset_global_tiny_random_graphs(G):
    gw, ctx = G
    cases = _tiny_cases(5502, 2000)
    g, base = union_graph([c[:4] for c in cases])
    say(f"global form, {len(cases)} tiny graphs with start offsets, one launch")
    graph = gw.Graph.of(ctx, g)
    try:
        seq, off = reads_of([c[2] for c in cases])
        res, paths = gw.align(ctx, graph, seq, off, np.array([c[3] + b for c, b in zip(cases, base)], np.int32),
                              start_off=np.array([c[4] for c in cases], np.int32),
                              v_end=np.array([c[5] + b for c, b in zip(cases, base)], np.int32),
                              path_cap=int(off[-1]) * 4 + 256 * len(cases))
    finally:
        graph.close()
    n_unreach = 0
    for i, (labels, edges, q, vs, j0, ve) in enumerate(cases):
        d = O.dp_dense_at((labels, edges), q, vs, j0, ve)[0]
        r = res[i]
        if d < 0:
            n_unreach += 1
            assert r["status"] == gw.ST_UNREACHABLE and r["dist"] == -1, i
            continue
        wf = O.gwf((labels, edges), q, vs, v_e=ve, j0=j0)
        assert (r["status"], r["dist"], r["end_v"] - base[i], r["end_off"], r["work"]) == \
            (0, d, ve, len(labels[ve]), wf["work"]), (i, labels, edges, q, vs, j0, ve)
        p = paths[i]
        assert p[0] == vs + base[i] and p[-1] == ve + base[i] and O.is_walk(g, p)
        assert O.ed_global(q, _spell_from(g, p, j0, len(labels[ve]))) == d
    assert 100 < n_unreach < len(cases) - 500


def test_start_offset_cfg1_exact_pruned_and_cigar(G):
    gw, ctx = G
    g, r = synth.cfg1()
    qs = [r.read(i) for i in range(r.n)]
    rng = np.random.default_rng(5503)
    j0 = np.array([int(rng.integers(0, g.seg_off[v + 1] - g.seg_off[v] + 1)) for v in r.v_start], np.int32)
    say("cfg1 reads with start offsets: exact + CIGAR, Algorithm 4")
    graph = gw.Graph.of(ctx, g)
    try:
        seq, off = reads_of(qs)
        n = r.n
        batch = gw.upload_reads(ctx, seq, off, np.asarray(r.v_start, np.int32))
        out = gw.alloc_out(ctx, n, int(off[-1]) * 2 + 256 * n)
        so = ctx.torch.from_numpy(j0).to(ctx.tdev)
        gw.step_dev(ctx, graph, batch, out, gw.opts(), None, so)
        res, path, _ = gw.fetch(out, n)
        ops, coff, clen = gw.cigar_dev(ctx, graph, batch, out)
        for i in range(n):
            d, ev, ej = O.dp_dense_at(g, qs[i], int(r.v_start[i]), int(j0[i]))
            ref = O.gwf(g, qs[i], int(r.v_start[i]), j0=int(j0[i]))
            x = res[i]
            assert (x["status"], x["dist"], x["end_v"], x["end_off"], x["work"]) == (0, d, ev, ej, ref["work"]), i
            p = path[x["path_off"]:x["path_off"] + x["path_len"]]
            T = _spell_from(g, p, int(j0[i]), ej)
            assert clen[i] >= 0 and refs.cigar_cost(qs[i], T, ops[coff[i]:coff[i] + clen[i]]) == d, i
        for a in (8, 30):
            res2, _ = gw.align(ctx, graph, seq, off, np.asarray(r.v_start, np.int32),
                               gw.opts(prune=gw.PRUNE_HEURISTIC, a_diff=a), start_off=j0)
            for i in range(n):
                ref = O.gwf(g, qs[i], int(r.v_start[i]), a_diff=a, j0=int(j0[i]))
                assert (res2[i]["dist"], res2[i]["end_v"], res2[i]["end_off"], res2[i]["work"]) == \
                    (ref["dist"], ref["end_v"], ref["end_j"], ref["work"]), (i, a)
    finally:
        graph.close()


def test_start_offset_out_of_range_is_a_per_query_status(G):
    gw, ctx = G
    g = synth.Graph.from_labels(["ACGT", "TT"], [(0, 1)])
    graph = gw.Graph.of(ctx, g)
    try:
        say("start offsets out of range")
        seq, off = reads_of([b"GTTT", b"GT", b"TT", b""])
        res, paths = gw.align(ctx, graph, seq, off, np.zeros(4, np.int32),
                              start_off=np.array([2, 5, 4, -1], np.int32))
        assert (res[0]["status"], res[0]["dist"], res[0]["end_v"], res[0]["end_off"]) == (0, 0, 1, 2)
        assert list(paths[0]) == [0, 1]
        assert res[1]["status"] == gw.ST_BAD_INPUT and res[3]["status"] == gw.ST_BAD_INPUT
        assert (res[2]["status"], res[2]["dist"], res[2]["end_v"], res[2]["end_off"]) == (0, 0, 1, 2)
    finally:
        graph.close()


def test_start_window_tiny_random_graphs(G):
    """Free start windows j0..j1 (both forms): distance, end and work
    bit-exact against the oracle; the traced walk starts inside the window,
    and re-scored from there it costs the distance."""
    gw, ctx = G
    rng = np.random.default_rng(5504)
    cases = []
    for _ in range(2000):
        labels, edges, q, vs = refs.random_case(rng, n_vtx=int(rng.integers(1, 7)),
                                                max_label=40 if rng.random() < 0.2 else 6, p_edge=0.35,
                                                qlen=int(rng.integers(0, 30)))
        L = len(labels[vs])
        j0 = int(rng.integers(0, L + 1))
        cases.append((labels, edges, q, vs, j0, int(rng.integers(j0, L + 1)), int(rng.integers(0, len(labels)))))
    g, base = union_graph([c[:4] for c in cases])
    graph = gw.Graph.of(ctx, g)
    try:
        seq, off = reads_of([c[2] for c in cases])
        vs_all = np.array([c[3] + b for c, b in zip(cases, base)], np.int32)
        j0s = np.array([c[4] for c in cases], np.int32)
        j1s = np.array([c[5] for c in cases], np.int32)
        say("start windows, extension form")
        res, paths = gw.align(ctx, graph, seq, off, vs_all, start_off=j0s, start_hi=j1s,
                              path_cap=int(off[-1]) * 4 + 256 * len(cases))
        say("start windows, global form")
        resg, pathsg = gw.align(ctx, graph, seq, off, vs_all, start_off=j0s, start_hi=j1s,
                                v_end=np.array([c[6] + b for c, b in zip(cases, base)], np.int32),
                                path_cap=int(off[-1]) * 4 + 256 * len(cases))
    finally:
        graph.close()
    for i, (labels, edges, q, vs, j0, j1, ve) in enumerate(cases):
        d, ev, ej = O.dp_dense_at((labels, edges), q, vs, j0, j1=j1)
        wf = O.gwf((labels, edges), q, vs, j0=j0, j1=j1)
        r = res[i]
        assert (r["status"], r["dist"], r["end_v"] - base[i], r["end_off"], r["work"]) == \
            (0, d, ev, ej, wf["work"]), (i, labels, edges, q, vs, j0, j1)
        so = int(r["start_off"])
        p = paths[i]
        assert j0 <= so <= j1 and p[0] == vs + base[i] and O.is_walk(g, p)
        assert O.ed_global(q, _spell_from(g, p, so, ej)) == d
        dg = O.dp_dense_at((labels, edges), q, vs, j0, ve, j1=j1)[0]
        rg = resg[i]
        if dg < 0:
            assert rg["status"] == gw.ST_UNREACHABLE, i
            continue
        wg = O.gwf((labels, edges), q, vs, v_e=ve, j0=j0, j1=j1)
        assert (rg["status"], rg["dist"], rg["end_v"] - base[i], rg["work"]) == (0, dg, ve, wg["work"]), i
        sg = int(rg["start_off"])
        assert j0 <= sg <= j1
        assert O.ed_global(q, _spell_from(g, pathsg[i], sg, len(labels[ve]))) == dg


def test_start_window_longer_than_the_list_reruns(G):
    """A window wider than the first tier's list capacity restarts on larger
    tiers and still gives the oracle's answer."""
    gw, ctx = G
    rng = np.random.default_rng(5505)
    lab = "".join("ACGT"[x] for x in rng.integers(0, 4, size=3000))
    labels, edges = [lab, "ACGTTGCA"], [(0, 1)]
    g = synth.Graph.from_labels(labels, edges)
    qs = [lab[2500:2600].encode() + b"ACGT", lab[10:60].encode(), lab[2990:].encode() + b"ACGTT"]
    c2 = gw.Context(0)
    c2.config(list_cap=1024)
    graph = gw.Graph.of(c2, g)
    try:
        say("window of 3,001 starts, list capacity 1,024")
        seq, off = reads_of(qs)
        res, paths = gw.align(c2, graph, seq, off, np.zeros(3, np.int32), start_off=np.zeros(3, np.int32),
                              start_hi=np.full(3, 3000, np.int32))
        for i, q in enumerate(qs):
            assert (res[i]["status"], res[i]["dist"], res[i]["end_v"], res[i]["end_off"]) == \
                (0,) + O.dp_dense_at((labels, edges), q, 0, 0, j1=3000), i
        assert [int(x) for x in res["start_off"]] == [2500, 10, 2990]
        assert c2.stats()["reruns"] >= 3
    finally:
        graph.close()
        c2.close()
