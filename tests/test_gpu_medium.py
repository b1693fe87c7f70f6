"""GPU parity on medium random graphs, between the tiny-graph tests and the
full workloads: 20-200 vertices with labels of 1-400 bases, bubbles, back
edges and self-loops (cycles), queries of 50-3,000 bases spelled along random
walks with 0-12% errors, so that wavefronts span several batches of the
workgroup and crossings go around cycles.  Exact runs in both forms:
distance, end and work bit-exact against the dense oracle and the
Algorithms 1-4 transcription, walks re-scored; Algorithm 4 against its
transcription; CIGARs re-scored."""
import numpy as np
import pytest

import oracle as O
from tests import refs
from tests.test_gpu_parity import union_graph, reads_of

pytestmark = pytest.mark.gpu

N_CASES = 150


def say(msg):
    print(f"[gpu-medium] {msg}", flush=True)


@pytest.fixture(scope="module")
def G(gpu_lib):
    ctx = gpu_lib.Context(0)
    yield gpu_lib, ctx
    ctx.close()


@pytest.fixture(scope="module")
def cases():
    rng = np.random.default_rng(8100)
    cs = [refs.medium_case(rng) for _ in range(N_CASES)]
    g, base = union_graph([c[:4] for c in cs])
    return cs, g, base


def _run(gw, ctx, g, base, cs, o, form, cigar=False):
    graph = gw.Graph.of(ctx, g)
    try:
        seq, off = reads_of([c[2] for c in cs])
        n = len(cs)
        batch = gw.upload_reads(ctx, seq, off, np.array([c[3] + b for c, b in zip(cs, base)], np.int32))
        out = gw.alloc_out(ctx, n, int(off[-1]) * 4 + 256 * n)
        ve = None
        if form == "global":
            ve = ctx.torch.from_numpy(np.array([c[4] + b for c, b in zip(cs, base)], np.int32)).to(ctx.tdev)
        gw.step_dev(ctx, graph, batch, out, o, ve)
        res, path, _ = gw.fetch(out, n)
        cig = gw.cigar_dev(ctx, graph, batch, out) if cigar else None
        return res, path, cig
    finally:
        graph.close()


@pytest.mark.parametrize("form", ["extension", "global"])
def test_medium_exact(G, cases, form):
    gw, ctx = G
    cs, g, base = cases
    say(f"{form}: {len(cs)} medium graphs, exact")
    res, path, _ = _run(gw, ctx, g, base, cs, gw.opts(), form)
    for i, (labels, edges, q, vs, vl) in enumerate(cs):
        ve = vl if form == "global" else -1
        d, ev, ej = O.dp_dense_at((labels, edges), q, vs, 0, ve)
        wf = O.gwf((labels, edges), q, vs, v_e=ve)
        r = res[i]
        assert (r["status"], r["dist"], r["end_v"] - base[i], r["end_off"], r["work"]) == \
            (0, d, ev, ej, wf["work"]), (form, i)
        p = path[r["path_off"]:r["path_off"] + r["path_len"]]
        assert p[0] == vs + base[i] and p[-1] == ev + base[i] and O.is_walk(g, p)
        assert O.ed_global(q, O.spell_walk(g, p, ej)) == d


@pytest.mark.parametrize("form", ["extension", "global"])
def test_medium_algorithm_4(G, cases, form):
    gw, ctx = G
    cs, g, base = cases
    a = 20
    say(f"{form}: {len(cs)} medium graphs, Algorithm 4 a_diff {a}")
    res, path, _ = _run(gw, ctx, g, base, cs, gw.opts(prune=gw.PRUNE_HEURISTIC, a_diff=a), form)
    for i, (labels, edges, q, vs, vl) in enumerate(cs):
        ve = vl if form == "global" else -1
        wf = O.gwf((labels, edges), q, vs, v_e=ve, a_diff=a)
        r = res[i]
        if wf["status"] != 0:        # pruning emptied the wavefront before the end vertex
            assert wf["status"] == 2 and r["status"] == gw.ST_UNREACHABLE, (form, i)
            continue
        assert (r["dist"], r["end_v"] - base[i], r["end_off"], r["work"]) == \
            (wf["dist"], wf["end_v"], wf["end_j"], wf["work"]), (form, i)
        # the walk is a witness: its best alignment costs between d* and the distance
        p = path[r["path_off"]:r["path_off"] + r["path_len"]]
        e = O.ed_global(q, O.spell_walk(g, p, int(r["end_off"])))
        assert O.dp_dense_at((labels, edges), q, vs, 0, ve)[0] <= e <= r["dist"], (form, i)


@pytest.mark.parametrize("form", ["extension", "global"])
def test_medium_cigar(G, cases, form):
    gw, ctx = G
    cs, g, base = cases
    say(f"{form}: {len(cs)} medium graphs, exact, then CIGARs")
    res, path, (ops, coff, clen) = _run(gw, ctx, g, base, cs, gw.opts(), form, cigar=True)
    for i, (labels, edges, q, vs, vl) in enumerate(cs):
        r = res[i]
        assert r["status"] == 0 and clen[i] >= 0, (form, i)
        p = path[r["path_off"]:r["path_off"] + r["path_len"]]
        T = O.spell_walk(g, p, int(r["end_off"]))
        assert refs.cigar_cost(q, T, ops[coff[i]:coff[i] + clen[i]]) == r["dist"], (form, i)


@pytest.mark.parametrize("form", ["extension", "global"])
def test_medium_clip_and_windows(G, form):
    """Free end gap in the query (e = 40) on the medium graphs with random
    tails of 0-29 bases appended and, for half the queries, a free start
    window: distance, end, clip and work bit-exact, the walk starts inside
    the window, CIGARs end with the clip."""
    gw, ctx = G
    rng = np.random.default_rng(8101)
    cs = []
    for _ in range(N_CASES):
        labels, edges, q, vs, vl = refs.medium_case(rng)
        q = q + bytes(b"ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(0, 30))))
        L = len(labels[vs])
        j0 = int(rng.integers(0, L + 1)) if rng.random() < 0.5 else 0
        j1 = int(rng.integers(j0, L + 1)) if rng.random() < 0.5 else j0
        cs.append((labels, edges, q, vs, vl, j0, j1))
    g, base = union_graph([c[:4] for c in cs])
    e = 40
    say(f"{form}: {len(cs)} medium graphs with tails, e = {e}, start windows, then CIGARs")
    graph = gw.Graph.of(ctx, g)
    try:
        seq, off = reads_of([c[2] for c in cs])
        n = len(cs)
        dev = lambda x: ctx.torch.from_numpy(np.ascontiguousarray(x, np.int32)).to(ctx.tdev)
        batch = gw.upload_reads(ctx, seq, off, np.array([c[3] + b for c, b in zip(cs, base)], np.int32))
        out = gw.alloc_out(ctx, n, int(off[-1]) * 4 + 256 * n)
        ve = dev([c[4] + b for c, b in zip(cs, base)]) if form == "global" else None
        gw.step_dev(ctx, graph, batch, out, gw.opts(query_end_free=e), ve, dev([c[5] for c in cs]),
                    dev([c[6] for c in cs]))
        res, path, _ = gw.fetch(out, n)
        ops, coff, clen = gw.cigar_dev(ctx, graph, batch, out)
    finally:
        graph.close()
    n_clip = 0
    for i, (labels, edges, q, vs, vl, j0, j1) in enumerate(cs):
        vee = vl if form == "global" else -1
        ee = min(e, len(q))
        d, ev, ej, clip = O.dp_dense_clip((labels, edges), q, vs, ee, j0=j0, j1=j1, v_e=vee)
        wf = O.gwf((labels, edges), q, vs, j0=j0, j1=j1, v_e=vee, e=ee)
        r = res[i]
        assert (r["status"], r["dist"], r["end_v"] - base[i], r["end_off"], r["clip"], r["work"]) == \
            (0, d, ev, ej, clip, wf["work"]), (form, i)
        n_clip += clip > 0
        so = int(r["start_off"])
        p = path[r["path_off"]:r["path_off"] + r["path_len"]]
        assert j0 <= so <= j1 and p[0] == vs + base[i] and O.is_walk(g, p)
        T = O.spell_walk(g, p, ej)[so:]
        assert O.ed_global(q[:len(q) - clip], T) == d
        w = ops[coff[i]:coff[i] + clen[i]]
        assert clen[i] >= 0 and refs.cigar_cost(q, T, w) == d
        if clip:
            assert (int(w[-1]) & 15) == 4 and int(w[-1]) >> 4 == clip
    assert n_clip > N_CASES // 3


@pytest.mark.parametrize("e", [0, 20])
def test_medium_walk_end_free(G, e):
    """Global form with a free end gap in the walk (opts.walk_end_free): the
    walk may end anywhere inside v_e.  Medium graphs whose queries stop
    part-way through their last vertex, start windows on half of them, with
    and without a free end gap in the query: distance, end, clip and work
    bit-exact against the dense oracle and the Algorithms 1-4 transcription,
    walks ending in v_e re-scored, CIGARs re-scored."""
    gw, ctx = G
    rng = np.random.default_rng(8102 + e)
    cs = []
    for _ in range(N_CASES):
        labels, edges, q, vs, vl = refs.medium_case(rng)
        L = len(labels[vs])
        j0 = int(rng.integers(0, L + 1)) if rng.random() < 0.5 else 0
        j1 = int(rng.integers(j0, L + 1)) if rng.random() < 0.5 else j0
        cs.append((labels, edges, q, vs, vl, j0, j1))
    g, base = union_graph([c[:4] for c in cs])
    say(f"{len(cs)} medium graphs, global form, walk end free, e = {e}, then CIGARs")
    graph = gw.Graph.of(ctx, g)
    try:
        seq, off = reads_of([c[2] for c in cs])
        n = len(cs)
        dev = lambda x: ctx.torch.from_numpy(np.ascontiguousarray(x, np.int32)).to(ctx.tdev)
        batch = gw.upload_reads(ctx, seq, off, np.array([c[3] + b for c, b in zip(cs, base)], np.int32))
        out = gw.alloc_out(ctx, n, int(off[-1]) * 4 + 256 * n)
        gw.step_dev(ctx, graph, batch, out, gw.opts(query_end_free=e, walk_end_free=True),
                    dev([c[4] + b for c, b in zip(cs, base)]), dev([c[5] for c in cs]), dev([c[6] for c in cs]))
        res, path, _ = gw.fetch(out, n)
        ops, coff, clen = gw.cigar_dev(ctx, graph, batch, out)
    finally:
        graph.close()
    n_inside = 0
    for i, (labels, edges, q, vs, ve, j0, j1) in enumerate(cs):
        ee = min(e, len(q))
        d, ev, ej, clip = O.dp_dense_clip((labels, edges), q, vs, ee, j0, j1, ve, wfree=True)
        wf = O.gwf((labels, edges), q, vs, v_e=ve, j0=j0, j1=j1, e=ee, wfree=True)
        r = res[i]
        assert (r["status"], r["dist"], r["end_v"] - base[i], r["end_off"], r["clip"], r["work"]) == \
            (0, d, ev, ej, clip, wf["work"]), i
        n_inside += ej < len(labels[ve])
        so = int(r["start_off"])
        p = path[r["path_off"]:r["path_off"] + r["path_len"]]
        assert j0 <= so <= j1 and p[0] == vs + base[i] and p[-1] == ve + base[i] and O.is_walk(g, p)
        T = O.spell_walk(g, p, ej)[so:]
        assert O.ed_global(q[:len(q) - clip], T) == d
        assert clen[i] >= 0 and refs.cigar_cost(q, T, ops[coff[i]:coff[i] + clen[i]]) == d
    assert n_inside > N_CASES // 2


@pytest.mark.parametrize("form", ["extension", "global"])
def test_medium_learned_prune(gpu_lib, cases, form):
    """The trained keep/drop network on the medium graphs, both forms: every
    query finishes (or its end vertex is reported unreachable when pruning
    emptied the wavefront), the distance is never below the exact one, the
    traced walk is a witness between the two, and the network with every
    diagonal kept (threshold -inf, no gate) reproduces the exact run."""
    from paper_2206_13574_amd import train_prune
    gw = gpu_lib
    cs, g, base = cases
    W = train_prune.load()
    ctx = gw.Context(0)
    try:
        ctx.mlp_load(W["w_bf16"], W["scale"])
        say(f"{form}: {len(cs)} medium graphs, learned pruning")
        res, path, _ = _run(gw, ctx, g, base, cs, gw.opts(prune=gw.PRUNE_LEARNED, keep_threshold=W["tau"],
                                                          mlp_gate=W["gate"], mlp_period=W["period"]), form)
        keep_all, _, _ = _run(gw, ctx, g, base, cs, gw.opts(prune=gw.PRUNE_LEARNED, keep_threshold=-1e30,
                                                            mlp_gate=0, mlp_period=1), form)
    finally:
        ctx.close()
    over = 0
    for i, (labels, edges, q, vs, vl) in enumerate(cs):
        ve = vl if form == "global" else -1
        d, ev, ej = O.dp_dense_at((labels, edges), q, vs, 0, ve)
        wf = O.gwf((labels, edges), q, vs, v_e=ve)
        assert (keep_all[i]["status"], keep_all[i]["dist"], keep_all[i]["end_v"] - base[i],
                keep_all[i]["end_off"], keep_all[i]["work"]) == (0, d, ev, ej, wf["work"]), (form, i)
        r = res[i]
        if r["status"] == gw.ST_UNREACHABLE:
            assert form == "global", i
            over += 1
            continue
        assert r["status"] == 0 and r["dist"] >= d, (form, i)
        over += r["dist"] > d
        p = path[r["path_off"]:r["path_off"] + r["path_len"]]
        e = O.ed_global(q, O.spell_walk(g, p, int(r["end_off"])))
        assert d <= e <= r["dist"], (form, i)
    say(f"{form}: {over} of {len(cs)} queries above the exact distance")
