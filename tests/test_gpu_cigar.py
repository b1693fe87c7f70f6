"""GPU base-level alignment along the traced walks (gwfa_cigar_dev): every
CIGAR aligns the query to its walk's string exactly and costs the reported
distance (exact runs) or at most it (pruned runs)."""
import numpy as np
import pytest

import oracle as O
from paper_2206_13574_amd import synth
from tests import refs
from tests.test_gpu_parity import union_graph, reads_of

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-cigar] {msg}", flush=True)


@pytest.fixture(scope="module")
def G(gpu_lib):
    ctx = gpu_lib.Context(0)
    yield gpu_lib, ctx
    ctx.close()


def _align_and_cigar(gw, ctx, g, seq, off, vs, o, v_end=None):
    graph = gw.Graph.of(ctx, g)
    try:
        n = len(off) - 1
        batch = gw.upload_reads(ctx, seq, off, vs)
        out = gw.alloc_out(ctx, n, int(off[-1]) * 2 + 256 * n)
        ve = None if v_end is None else ctx.torch.from_numpy(np.asarray(v_end, dtype=np.int32)).to(ctx.tdev)
        gw.step_dev(ctx, graph, batch, out, o, ve)
        res, path, _ = gw.fetch(out, n)
        ops, coff, clen = gw.cigar_dev(ctx, graph, batch, out)
        return res, path, ops, coff, clen
    finally:
        graph.close()


def _check(g, qs, res, path, ops, coff, clen, dstar, exact=True):
    """Every CIGAR aligns its query to its walk's string exactly; exact runs
    cost the oracle's distance d*, pruned runs at most their reported
    distance, which is never below d*."""
    n_ok = 0
    for i, q in enumerate(qs):
        r = res[i]
        if r["status"] != 0:
            assert clen[i] == -1
            continue
        n_ok += 1
        p = path[r["path_off"]:r["path_off"] + r["path_len"]]
        t = O.spell_walk(g, p, int(r["end_off"]))
        cost = refs.cigar_cost(q, t, ops[coff[i]:coff[i] + clen[i]])
        if exact:
            assert cost == dstar[i] == r["dist"], (i, cost, dstar[i], int(r["dist"]))
        else:
            assert cost <= r["dist"] and r["dist"] >= dstar[i], (i, cost, dstar[i], int(r["dist"]))
    return n_ok


@pytest.mark.parametrize("form", ["extension", "global"])
def test_cigar_tiny_random(G, form):
    gw, ctx = G
    rng = np.random.default_rng(9401)
    cases = []
    for _ in range(1500):
        labels, edges, q, vs = refs.random_case(rng, n_vtx=int(rng.integers(1, 7)), max_label=5, p_edge=0.35,
                                                qlen=int(rng.integers(0, 40)))
        cases.append((labels, edges, q, vs, int(rng.integers(0, len(labels)))))
    g, base = union_graph([c[:4] for c in cases])
    qs = [c[2] for c in cases]
    seq, off = reads_of(qs)
    vs = np.array([c[3] + b for c, b in zip(cases, base)], np.int32)
    ve = np.array([c[4] + b for c, b in zip(cases, base)], np.int32) if form == "global" else None
    say(f"{form}: {len(cases)} tiny graphs")
    res, path, ops, coff, clen = _align_and_cigar(gw, ctx, g, seq, off, vs, gw.opts(), ve)
    if form == "global":
        dstar = [O.dp_dense_global((c[0], c[1]), c[2], c[3], c[4]) for c in cases]
        for i, d in enumerate(dstar):   # an unreachable end vertex is a status, and gets no CIGAR
            assert (res[i]["status"] == gw.ST_UNREACHABLE) == (d < 0), i
    else:
        dstar = [O.dp_dense((c[0], c[1]), c[2], c[3])[0] for c in cases]
    assert _check(g, qs, res, path, ops, coff, clen, dstar) > 800


def test_cigar_cfg2_subset_exact_and_pruned(G):
    gw, ctx = G
    g, r = synth.cfg2(n_reads=600)
    qs = [r.read(i) for i in range(r.n)]
    dstar = O.dp_batch(g, r.seq, r.off, r.v_start, r.n_edits)[:, 0]
    assert (dstar >= 0).all()
    for o, exact in ((gw.opts(), True), (gw.opts(prune=gw.PRUNE_HEURISTIC, a_diff=30), False)):
        say(f"cfg2[:600] prune={o.prune}")
        res, path, ops, coff, clen = _align_and_cigar(gw, ctx, g, r.seq, r.off, r.v_start, o)
        assert _check(g, qs, res, path, ops, coff, clen, dstar, exact) == r.n
