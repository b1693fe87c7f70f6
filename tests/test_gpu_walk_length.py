"""GPU parity of the walk length W~ of Algorithm 4 (Section 2.5), entry by
entry.

The trace dump writes one record per wavefront entry that survives the
score's pruning pass: (score, v, k, offset, W~).  For every query and every
score before the end, that set must equal the oracle's extended entries of
the same score (orc_gwf, whose W~ is pinned on the CPU: a real walk length
at no more than the score, and the tie rules against an independent
implementation) after Algorithm 4's keep rule (a = i + W~; when the largest
a exceeds a_diff, keep a_max - a < a_diff).  Exact runs keep every entry.
Tiny random graphs with cycles and self-loops, and medium graphs with indel
bubbles, back edges and self-loops, where walks of different lengths meet.
Bar: the sets equal, bit for bit, and so do distance and end."""
import numpy as np
import pytest

import oracle as O
from tests import refs
from tests.test_gpu_parity import reads_of, union_graph

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-walk] {msg}", flush=True)


@pytest.fixture(scope="module")
def G(gpu_lib):
    ctx = gpu_lib.Context(0)
    yield gpu_lib, ctx
    ctx.close()


def kept_entries(ent: np.ndarray, dist: int, a_diff: int) -> list:
    """The oracle's extended entries (score, v, k, off, W~) of scores before
    `dist` that Algorithm 4 keeps, sorted."""
    out = []
    for s in range(dist):
        e = ent[ent[:, 0] == s]
        if a_diff > 0 and len(e):
            a = e[:, 2].astype(np.int64) + e[:, 3] + e[:, 4]
            amax = max(int(a.max()), 0)
            if amax > a_diff:
                e = e[amax - a < a_diff]
        out += [tuple(x) for x in e.tolist()]
    return sorted(out)


def compare(gw, ctx, cases, a_diff: int):
    g, base = union_graph(cases)
    graph = gw.Graph.of(ctx, g)
    seq, off = reads_of([c[2] for c in cases])
    vs = np.asarray([c[3] + b for c, b in zip(cases, base)], dtype=np.int32)
    o = gw.opts(prune=gw.PRUNE_HEURISTIC if a_diff else gw.PRUNE_NONE, a_diff=a_diff, traceback=False)
    try:
        res, d, produced = gw.align_dump(ctx, graph, seq, off, vs, o, dump_cap=1 << 22)
    finally:
        graph.close()
    assert produced <= 1 << 22
    assert (res["status"] == 0).all()
    rows = np.stack([d["read"], d["score"], d["v"], d["k"], d["off"], d["W"]], 1)
    rows = rows[np.lexsort(rows.T[::-1])]
    starts = np.searchsorted(rows[:, 0], np.arange(len(cases) + 1))
    n_entries = 0
    for i, (labels, edges, q, v_s) in enumerate(cases):
        ref = O.gwf((labels, edges), q, v_s, a_diff=a_diff, entries_cap=1 << 22)
        assert ref["entries_total"] == len(ref["entries"])
        got = (int(res[i]["dist"]), int(res[i]["end_v"]) - base[i], int(res[i]["end_off"]))
        assert got == (ref["dist"], ref["end_v"], ref["end_j"]), (i, a_diff)
        mine = rows[starts[i]:starts[i + 1], 1:].copy()
        mine[:, 1] -= base[i]
        want = kept_entries(ref["entries"], ref["dist"], a_diff)
        assert sorted(map(tuple, mine.tolist())) == want, (i, a_diff, labels, edges, q, v_s)
        n_entries += len(want)
    return n_entries


def test_walk_lengths_tiny_random_graphs(G):
    gw, ctx = G
    rng = np.random.default_rng(5101)
    cases = [refs.random_case(rng, n_vtx=int(rng.integers(1, 8)), max_label=6, p_edge=float(rng.uniform(0.15, 0.5)),
                              qlen=int(rng.integers(0, 50))) for _ in range(1500)]
    for a_diff in (0, 3, 8, 20):
        say(f"tiny random graphs: {len(cases)} cases, a_diff={a_diff}")
        n = compare(gw, ctx, cases, a_diff)
        assert n > 50000


def test_walk_lengths_medium_graphs(G):
    gw, ctx = G
    rng = np.random.default_rng(5102)
    cases = []
    for _ in range(30):
        labels, edges, q, vs, _ = refs.medium_case(rng)
        cases.append((labels, edges, q[:int(rng.integers(50, 800))], vs))
    for a_diff in (0, 10, 40):
        say(f"medium graphs: {len(cases)} cases, a_diff={a_diff}")
        n = compare(gw, ctx, cases, a_diff)
        assert n > (100000 if a_diff == 0 else 1000)
