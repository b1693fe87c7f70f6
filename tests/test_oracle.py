"""Pins for the CPU oracle against facts that the paper and plain
mathematics fix (no GPU needed).

* brute-force walk enumeration on tiny graphs, cycles and self-loops
  included (Def. 2.2: the optimum over all walks);
* single-path graphs reduce to pairwise edit distance (Section 2.2: the
  recurrence generalises the pairwise DP), end free in the target;
* invariants: 0 <= d* <= |q|; d* = 0 for queries a walk spells; prefix
  distances never drop and grow by at most one per base; d* <= injected edits;
* graph transforms: splitting labels into one-base chains (the
  string/char-labelled equivalence stated in Section 2.2), permuting vertex
  ids and cutting one label in two leave d* and the end set unchanged;
* the value-capped form equals the dense form;
* Algorithms 1-3 reach the Eq. 1 optimum and end; Algorithm 4 with a huge
  a_diff is exact and never beats the optimum otherwise; the work count
  respects the diagonal-length bound of Section 2.4;
* Algorithm 4 equals a pairwise wavefront with the same keep rule where every
  walk has the same length up to each base; elsewhere every walk length W~ is
  that of a walk aligning the consumed query at no more than the entry's
  score, and the tie rules between walks of different lengths agree with an
  independent implementation of them.
"""
import numpy as np
import pytest

import oracle as O
from paper_2206_13574_amd import synth
from tests import refs


# ---------------------------------------------------------------------------
# hand-worked cases (closed forms read off Eq. 1 by hand)
# ---------------------------------------------------------------------------
HAND = [
    # graph, query, v_s, d*, end(v, j)
    ((["ACG", "T", "A", "CC"], [(0, 1), (0, 2), (1, 3), (2, 3)]), b"ACGTCC", 0, 0, (3, 2)),
    ((["ACG", "T", "A", "CC"], [(0, 1), (0, 2), (1, 3), (2, 3)]), b"ACGACC", 0, 0, (3, 2)),
    # G instead of T/A at the bubble: one substitution; both arms tie, the
    # end cell (3,2) is the only end reached at cost 1
    ((["ACG", "T", "A", "CC"], [(0, 1), (0, 2), (1, 3), (2, 3)]), b"ACGGCC", 0, 1, (3, 2)),
    # empty query: distance 0 at (v_s, 0)
    ((["ACG", "T"], [(0, 1)]), b"", 0, 0, (0, 0)),
    # "TTT" against prefixes of "ACGT": the empty prefix costs 3 (insertions)
    # and no prefix does better (ed with "ACGT" is 3 too), so d* = 3 and the
    # start cell (0,0), which holds 3, is the smallest end cell
    ((["ACG", "T"], [(0, 1)]), b"TTT", 0, 3, (0, 0)),
    # self-loop: "AC" repeated; ACACAC spells 3 laps exactly.  The end of a
    # lap carries at zero cost onto (v_s, 0), which is an end cell of the same
    # value and sorts first
    ((["AC"], [(0, 0)]), b"ACACAC", 0, 0, (0, 0)),
    # self-loop with a missing base: ACAAC against ACACAC deletes one C
    ((["AC"], [(0, 0)]), b"ACAAC", 0, 1, (0, 0)),
    # without the loop the same query must insert past the label end
    ((["AC"], []), b"ACAAC", 0, 3, (0, 2)),
    # start vertex matters: same graph, start at 1
    ((["ACG", "T", "A", "CC"], [(0, 1), (0, 2), (1, 3), (2, 3)]), b"TCC", 1, 0, (3, 2)),
    # a query longer than every walk: the tail must be inserted
    ((["AC", "G"], [(0, 1)]), b"ACGTT", 0, 2, (1, 1)),
]


@pytest.mark.parametrize("case", HAND)
def test_hand_cases(case):
    g, q, vs, d, end = case
    assert O.dp_dense(g, q, vs)[:3] == (d, end[0], end[1])
    assert O.dp_capped(g, q, vs, len(q) + 1) == (d, end[0], end[1])
    r = O.gwf(g, q, vs)
    assert (r["dist"], r["end_v"], r["end_j"]) == (d, end[0], end[1])
    bd, bends = refs.brute_force(g[0], g[1], q, vs)
    assert bd == d and end in bends and end == min(bends)


# ---------------------------------------------------------------------------
# brute force on random tiny graphs
# ---------------------------------------------------------------------------
def test_brute_force_random_tiny():
    rng = np.random.default_rng(7)
    n_cases = 0
    for _ in range(400):
        labels, edges, q, vs = refs.random_case(rng, n_vtx=int(rng.integers(1, 6)), max_label=3,
                                                p_edge=0.35, qlen=int(rng.integers(0, 8)))
        bd, bends = refs.brute_force(labels, edges, q, vs)
        d, ev, ej, sweeps = O.dp_dense((labels, edges), q, vs)
        assert d == bd, (labels, edges, q, vs)
        assert (ev, ej) == min(bends), (labels, edges, q, vs, bends)
        assert sweeps <= len(labels) + 1
        n_cases += 1
    assert n_cases == 400


def test_brute_force_walk_spelled_queries():
    """Queries that a walk from (v_s,0) spells have distance 0 (and brute force
    agrees on the end)."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        labels, edges, _, vs = refs.random_case(rng, n_vtx=5, max_label=3, p_edge=0.35, qlen=0)
        q, _ = refs.spell_random_walk(rng, labels, edges, vs, int(rng.integers(1, 10)))
        d, ev, ej, _ = O.dp_dense((labels, edges), q, vs)
        assert d == 0
        bd, bends = refs.brute_force(labels, edges, q, vs)
        assert bd == 0 and (ev, ej) == min(bends)


# ---------------------------------------------------------------------------
# single-path graphs = pairwise edit distance, end free in the target
# ---------------------------------------------------------------------------
def test_chain_equals_semiglobal_ed():
    rng = np.random.default_rng(3)
    for _ in range(60):
        T = "".join("ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(1, 40))))
        cuts = sorted(set(rng.integers(1, len(T), size=int(rng.integers(0, 6))).tolist())) if len(T) > 1 else []
        pieces = [T[a:b] for a, b in zip([0] + cuts, cuts + [len(T)])]
        edges = [(i, i + 1) for i in range(len(pieces) - 1)]
        if rng.random() < 0.5:   # a mutated copy of a prefix
            q = bytearray(T[: int(rng.integers(0, len(T) + 1))].encode())
            for _ in range(int(rng.integers(0, 4))):
                if q and rng.random() < 0.5:
                    q[int(rng.integers(0, len(q)))] = ord("ACGT"[int(rng.integers(0, 4))])
                else:
                    q.insert(int(rng.integers(0, len(q) + 1)), ord("ACGT"[int(rng.integers(0, 4))]))
            q = bytes(q)
        else:
            q = "".join("ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(0, 30)))).encode()
        row = refs.semiglobal_ed_row(q, T.encode())
        dstar = int(row.min())
        p = int(np.argmin(row))           # smallest prefix length with the optimum
        starts = np.cumsum([0] + [len(x) for x in pieces])
        if p == 0:
            end = (0, 0)
        else:
            v = int(np.searchsorted(starts, p, side="left")) - 1
            end = (v, p - int(starts[v]))
        got = O.dp_dense((pieces, edges), q, 0)
        assert got[0] == dstar and got[1:3] == end, (pieces, q, row.tolist())
        assert O.gwf((pieces, edges), q, 0)["dist"] == dstar


def test_textbook_ed_against_library_pairwise():
    """The oracle's pairwise routines agree with the numpy textbook DP, and the
    banded form is exact within its band."""
    rng = np.random.default_rng(5)
    for _ in range(100):
        a = "".join("ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(0, 30)))).encode()
        b = "".join("ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(0, 30)))).encode()
        e = refs.ed(a, b)
        assert O.ed_global(a, b) == e
        for D in (0, 1, 3, 8, 40):
            assert O.ed_banded(a, b, D) == (e if e <= D else -1)


# ---------------------------------------------------------------------------
# invariants on the generated workloads
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def cfg1():
    return synth.cfg1()


def test_cfg1_invariants_and_capped_equals_dense(cfg1):
    g, r = cfg1
    for i in range(r.n):
        q = r.read(i)
        d, ev, ej, _ = O.dp_dense(g, q, int(r.v_start[i]))
        assert 0 <= d <= len(q)
        assert d <= int(r.n_edits[i])              # the generating walk aligns with that many edits
        assert O.dp_capped(g, q, int(r.v_start[i]), int(r.n_edits[i])) == (d, ev, ej)
        if d > 0:
            assert O.dp_capped(g, q, int(r.v_start[i]), d - 1)[0] == -1
        res = O.gwf(g, q, int(r.v_start[i]))
        assert (res["dist"], res["end_v"], res["end_j"]) == (d, ev, ej)


def test_prefix_distances_monotone(cfg1):
    """m_i = d*(q[1..i]) never decreases and grows by at most 1 per base."""
    g, r = cfg1
    q = r.read(0)[:120]
    m = [O.dp_dense(g, q[:i], int(r.v_start[0]))[0] for i in range(len(q) + 1)]
    steps = np.diff(m)
    assert ((steps == 0) | (steps == 1)).all()


def test_capped_equals_dense_random():
    rng = np.random.default_rng(21)
    for _ in range(300):
        labels, edges, q, vs = refs.random_case(rng, n_vtx=int(rng.integers(1, 8)), max_label=5,
                                                p_edge=0.3, qlen=int(rng.integers(0, 25)))
        d, ev, ej, _ = O.dp_dense((labels, edges), q, vs)
        for D in (d, d + 1, d + 5):
            assert O.dp_capped((labels, edges), q, vs, D) == (d, ev, ej)
        if d > 0:
            assert O.dp_capped((labels, edges), q, vs, d - 1)[0] == -1


def test_gwf_equals_dense_random():
    rng = np.random.default_rng(23)
    for _ in range(300):
        labels, edges, q, vs = refs.random_case(rng, n_vtx=int(rng.integers(1, 8)), max_label=5,
                                                p_edge=0.3, qlen=int(rng.integers(0, 25)))
        d, ev, ej, _ = O.dp_dense((labels, edges), q, vs)
        res = O.gwf((labels, edges), q, vs)
        assert (res["dist"], res["end_v"], res["end_j"]) == (d, ev, ej), (labels, edges, q, vs)


def test_char_split_invariance():
    rng = np.random.default_rng(31)
    for _ in range(150):
        labels, edges, q, vs = refs.random_case(rng, n_vtx=int(rng.integers(1, 6)), max_label=4,
                                                p_edge=0.35, qlen=int(rng.integers(0, 12)))
        bd, bends = refs.brute_force(labels, edges, q, vs)
        nl, ne, first, last, cmap = refs.char_split(labels, edges)
        d2, ev2, ej2, _ = O.dp_dense((nl, ne), q, first[vs])
        assert d2 == bd
        # the split graph's end set is the image of the original one
        mapped = {cmap[(v, j)] if j > 0 else (first[v], 0) for v, j in bends}
        bd2, bends2 = refs.brute_force(nl, ne, q, first[vs])
        assert bends2 == mapped
        assert (ev2, ej2) == min(bends2)


def test_vertex_permutation_invariance():
    rng = np.random.default_rng(37)
    for _ in range(150):
        labels, edges, q, vs = refs.random_case(rng, n_vtx=int(rng.integers(1, 7)), max_label=4,
                                                p_edge=0.3, qlen=int(rng.integers(0, 12)))
        bd, bends = refs.brute_force(labels, edges, q, vs)
        perm = rng.permutation(len(labels))        # old id -> new id
        nl = [None] * len(labels)
        for v, s in enumerate(labels):
            nl[perm[v]] = s
        ne = [(int(perm[a]), int(perm[b])) for a, b in edges]
        d2, ev2, ej2, _ = O.dp_dense((nl, ne), q, int(perm[vs]))
        assert d2 == bd
        assert (ev2, ej2) == min((int(perm[v]), j) for v, j in bends)


def test_label_cut_invariance():
    """Cutting one label in two (the pieces joined by an edge, out-edges moved
    to the second piece) leaves d* unchanged."""
    rng = np.random.default_rng(41)
    for _ in range(150):
        labels, edges, q, vs = refs.random_case(rng, n_vtx=int(rng.integers(1, 6)), max_label=6,
                                                p_edge=0.3, qlen=int(rng.integers(0, 14)))
        v = int(rng.integers(0, len(labels)))
        if len(labels[v]) < 2:
            continue
        c = int(rng.integers(1, len(labels[v])))
        nv = len(labels)
        nl = labels[:v] + [labels[v][:c]] + labels[v + 1:] + [labels[v][c:]]
        ne = []
        for a, b in edges:
            ne.append((nv if a == v else a, b))
        ne.append((v, nv))
        d = O.dp_dense((labels, edges), q, vs)[0]
        assert O.dp_dense((nl, ne), q, vs)[0] == d


# ---------------------------------------------------------------------------
# Algorithm 4 and work counts
# ---------------------------------------------------------------------------
def test_prune_huge_a_diff_is_exact_and_never_better(cfg1):
    g, r = cfg1
    for i in range(0, r.n, 5):
        q = r.read(i)
        vs = int(r.v_start[i])
        ex = O.gwf(g, q, vs)
        big = O.gwf(g, q, vs, a_diff=10 ** 8)
        assert (big["dist"], big["end_v"], big["end_j"], big["work"]) == \
               (ex["dist"], ex["end_v"], ex["end_j"], ex["work"])
        for a_diff in (5, 20, 60, 200):
            pr = O.gwf(g, q, vs, a_diff=a_diff)
            assert pr["status"] == 0 and pr["dist"] >= ex["dist"]
            assert pr["work"] <= ex["work"] or pr["dist"] > ex["dist"]


def test_work_bound_section_2_4(cfg1):
    """Each diagonal is updated at most (its length + 1) times, so the total
    wavefront work is at most the number of diagonals times (max |v| + 1)
    plus one per crossing."""
    g, r = cfg1
    lens = np.diff(g.seg_off)
    for i in range(0, r.n, 10):
        res = O.gwf(g, r.read(i), int(r.v_start[i]), counts_cap=4096)
        assert sum(res["counts"]) == res["work"]
        assert res["work"] <= res["diagonals"] * (int(lens.max()) + 1)


def test_pairwise_wavefront_counts():
    """On a single-vertex graph the wavefront is the pairwise one: at score s
    it holds at most 2s+1 diagonals."""
    rng = np.random.default_rng(2)
    T = "".join("ACGT"[x] for x in rng.integers(0, 4, size=300))
    q = bytearray(T[:250].encode())
    for _ in range(12):
        q[int(rng.integers(0, len(q)))] = ord("ACGT"[int(rng.integers(0, 4))])
    res = O.gwf(([T], []), bytes(q), 0, counts_cap=1000)
    for s, c in enumerate(res["counts"]):
        assert c <= 2 * s + 1


def test_reverse_labels_consistency(cfg1):
    """R_{0,v_s,0} of the reverse recurrence equals d* of the forward one."""
    import ctypes
    g, r = cfg1
    G = O.OGraph.of(g)
    lib = O._load()
    for i in range(0, r.n, 10):
        q = np.frombuffer(r.read(i), dtype=np.uint8).copy()
        vs = int(r.v_start[i])
        ei = np.array([0], dtype=np.int32)
        ev = np.array([vs], dtype=np.int32)
        eo = np.array([0], dtype=np.int32)
        cost = np.zeros(1, dtype=np.int32)
        dst = np.zeros(1, dtype=np.int32)
        rc = lib.orc_rev_labels(*G._args(), O._ptr(q), len(q), vs, O._ptr(ei), O._ptr(ev), O._ptr(eo),
                                O._ptr(cost), 1, O._ptr(dst))
        assert rc == 0
        assert int(dst[0]) == O.dp_dense(g, q, vs)[0] == int(cost[0])


def test_reverse_labels_equal_forward_suffix_runs():
    """R(i, v, 0) is d* of the query suffix q[i+1..] started at (v, 0): the
    reverse recurrence pinned cell by cell against the forward oracle (itself
    pinned by brute force), on random cyclic graphs."""
    rng = np.random.default_rng(8101)
    lib = O._load()
    for case in range(60):
        g = synth.small_random_graph(rng, int(rng.integers(1, 6)), max_label=4, p_edge=0.35, cyclic=True)
        G = O.OGraph.of(g)
        q = "".join("ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(0, 9)))).encode()
        vs = int(rng.integers(0, g.n_vtx))
        ei = np.array([i for i in range(len(q) + 1) for v in range(g.n_vtx)], dtype=np.int32)
        ev = np.array([v for i in range(len(q) + 1) for v in range(g.n_vtx)], dtype=np.int32)
        eo = np.zeros(len(ei), dtype=np.int32)
        cost = np.zeros(len(ei), dtype=np.int32)
        dst = np.zeros(1, dtype=np.int32)
        qa = np.frombuffer(q, dtype=np.uint8).copy()
        assert lib.orc_rev_labels(*G._args(), O._ptr(qa), len(qa), vs, O._ptr(ei), O._ptr(ev), O._ptr(eo),
                                  O._ptr(cost), len(ei), O._ptr(dst)) == 0
        for e in range(len(ei)):
            assert int(cost[e]) == O.dp_dense(g, q[int(ei[e]):], int(ev[e]))[0], (case, e)


# ---------------------------------------------------------------------------
# global form (Definition 2.2 with an end vertex)
# ---------------------------------------------------------------------------
def test_global_chains_equal_textbook_edit_distance():
    """On a chain the global form is the pairwise edit distance between the
    query and the labels from v_s through v_e."""
    rng = np.random.default_rng(8201)
    for case in range(80):
        nv = int(rng.integers(1, 7))
        labels = ["".join("ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(1, 6)))) for _ in range(nv)]
        edges = [(i, i + 1) for i in range(nv - 1)]
        a = int(rng.integers(0, nv))
        b = int(rng.integers(a, nv))
        q = "".join("ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(0, 14)))).encode()
        want = refs.ed(q, "".join(labels[a:b + 1]).encode())
        assert O.dp_dense_global((labels, edges), q, a, b) == want, case
        assert O.gwf((labels, edges), q, a, v_e=b)["dist"] == want, case
        if a > 0:   # v_e before v_s on the chain: unreachable
            assert O.dp_dense_global((labels, edges), q, a, a - 1) == -1
            assert O.gwf((labels, edges), q, a, v_e=a - 1)["status"] == 2


def test_global_brute_force_random_tiny():
    """Random tiny graphs with cycles and self-loops against walk
    enumeration; the extension form's distance is never larger."""
    rng = np.random.default_rng(8202)
    n_reach = 0
    for case in range(300):
        labels, edges, q, v_s = refs.random_case(rng, n_vtx=int(rng.integers(1, 5)), max_label=3,
                                                 p_edge=0.35, qlen=int(rng.integers(0, 6)))
        v_e = int(rng.integers(0, len(labels)))
        want = refs.brute_force_global(labels, edges, q, v_s, v_e)
        got = O.dp_dense_global((labels, edges), q, v_s, v_e)
        assert got == want, (case, labels, edges, q, v_s, v_e)
        gw = O.gwf((labels, edges), q, v_s, v_e=v_e)
        assert (gw["dist"] if gw["status"] == 0 else -1) == want, case
        if want >= 0:
            n_reach += 1
            assert O.dp_dense((labels, edges), q, v_s)[0] <= want
    assert n_reach > 150


# ---------------------------------------------------------------------------
# walks that start inside the start vertex (a read seeded at offset j0)
# ---------------------------------------------------------------------------
START_HAND = [
    # graph, query, v_s, j0, d*, end(v, j)
    # "GTCC" from offset 2 of ACG: G, then the T arm, then CC
    ((["ACG", "T", "A", "CC"], [(0, 1), (0, 2), (1, 3), (2, 3)]), b"GTCC", 0, 2, 0, (3, 2)),
    # the same query from offset 0 must delete "AC" first (or insert)
    ((["ACG", "T", "A", "CC"], [(0, 1), (0, 2), (1, 3), (2, 3)]), b"GTCC", 0, 0, 2, (3, 2)),
    # empty query from offset 1: distance 0 at the start cell (0, 1)
    ((["ACG", "T"], [(0, 1)]), b"", 0, 1, 0, (0, 1)),
    # starting at the end of v_s: the walk goes on into the successor
    ((["ACG", "T"], [(0, 1)]), b"T", 0, 3, 0, (1, 1)),
    # self-loop from offset 1: "C" then a full lap "AC"; the lap's end cell
    # (0, 2) sorts before the zero-cost carry onto (0, 0), which is no end
    # cell when the walk starts at offset 1
    ((["AC"], [(0, 0)]), b"CAC", 0, 1, 0, (0, 2)),
]


@pytest.mark.parametrize("case", START_HAND)
def test_start_offset_hand_cases(case):
    g, q, vs, j0, d, end = case
    assert O.dp_dense_at(g, q, vs, j0) == (d, end[0], end[1])
    gw = O.gwf(g, q, vs, j0=j0)
    assert (gw["dist"], gw["end_v"], gw["end_j"]) == (d, end[0], end[1])


def test_start_offset_brute_force_random_tiny():
    """Random tiny graphs (cycles, self-loops) with a random start offset:
    the dense form and Algorithms 1-3 against walk enumeration from (v_s, j0),
    in extension mode (d* and an end from the enumerated end set) and in the
    global form."""
    rng = np.random.default_rng(6113)
    n_pos = 0
    for case in range(300):
        labels, edges, q, v_s = refs.random_case(rng, n_vtx=int(rng.integers(1, 5)), max_label=4,
                                                 p_edge=0.35, qlen=int(rng.integers(0, 7)))
        j0 = int(rng.integers(0, len(labels[v_s]) + 1))
        n_pos += j0 > 0
        g = (labels, edges)
        bd, bends = refs.brute_force(labels, edges, q, v_s, j0)
        d, ev, ej = O.dp_dense_at(g, q, v_s, j0)
        assert d == bd and (ev, ej) == min(bends), (case, labels, edges, q, v_s, j0)
        gw = O.gwf(g, q, v_s, j0=j0)
        assert (gw["dist"], gw["end_v"], gw["end_j"]) == (d, ev, ej), case
        v_e = int(rng.integers(0, len(labels)))
        want = refs.brute_force_global(labels, edges, q, v_s, v_e, j0)
        assert O.dp_dense_at(g, q, v_s, j0, v_e)[0] == want, (case, v_e)
        gg = O.gwf(g, q, v_s, v_e=v_e, j0=j0)
        assert (gg["dist"] if gg["status"] == 0 else -1) == want, case
    assert n_pos > 150


def test_start_offset_equals_cut_start_vertex():
    """Starting after j0 bases of v_s equals starting at offset 0 of a new
    vertex spelling the rest of v_s's label with v_s's out-edges (v_s itself
    stays for walks that come back to it); ends map (new, j) -> (v_s, j0 + j)
    and (new, 0) -> (v_s, j0)."""
    rng = np.random.default_rng(77)
    for case in range(200):
        labels, edges, q, v_s = refs.random_case(rng, n_vtx=int(rng.integers(1, 6)), max_label=6,
                                                 p_edge=0.3, qlen=int(rng.integers(0, 12)))
        if len(labels[v_s]) < 2:
            continue
        j0 = int(rng.integers(1, len(labels[v_s])))
        nv = len(labels)
        nl = labels + [labels[v_s][j0:]]
        ne = edges + [(nv, b) for a, b in edges if a == v_s]
        d, ev, ej = O.dp_dense_at((labels, edges), q, v_s, j0)
        d2, ev2, ej2, _ = O.dp_dense((nl, ne), q, nv)
        assert d2 == d, case
        # the new vertex sorts last; map its cells back before comparing
        # with the cells the original graph reaches at d*
        _, bends = refs.brute_force(labels, edges, q, v_s, j0)
        assert (ev, ej) in bends
        m = (v_s, j0 + ej2) if ev2 == nv else (ev2, ej2)
        assert m in bends, case


# ---------------------------------------------------------------------------
# a free leading gap in the start vertex: any start in j0..j1 at no cost
# ---------------------------------------------------------------------------
def test_start_window_hand_cases():
    g = (["ACGTACGG", "TT"], [(0, 1)])
    # "GGTT": the window 0..8 lets the walk start at offset 6 of vertex 0
    assert O.dp_dense_at(g, b"GGTT", 0, 0, j1=8) == (0, 1, 2)
    # from offset 0 only: the best prefix is "ACGT" (three substitutions), as
    # the textbook semi-global row of the chain's string says
    assert O.dp_dense_at(g, b"GGTT", 0, 0)[0] == 3 == int(refs.semiglobal_ed_row(b"GGTT", b"ACGTACGGTT").min())
    # a window that ends before the seed: the minimum over its four starts
    d = O.dp_dense_at(g, b"GGTT", 0, 0, j1=3)[0]
    assert d == min(O.dp_dense_at(g, b"GGTT", 0, j)[0] for j in range(4))
    gw = O.gwf(g, b"GGTT", 0, j0=0, j1=8)
    assert (gw["dist"], gw["end_v"], gw["end_j"]) == (0, 1, 2)


def test_start_window_brute_force_random_tiny():
    """Windows j0..j1 on random tiny graphs: the dense form and Algorithms
    1-3 against walk enumeration from every start of the window (extension
    mode: d* and the end; global form: the distance)."""
    rng = np.random.default_rng(771)
    n_win = 0
    for case in range(300):
        labels, edges, q, v_s = refs.random_case(rng, n_vtx=int(rng.integers(1, 5)), max_label=5,
                                                 p_edge=0.35, qlen=int(rng.integers(0, 7)))
        L = len(labels[v_s])
        j0 = int(rng.integers(0, L + 1))
        j1 = int(rng.integers(j0, L + 1))
        n_win += j1 > j0
        g = (labels, edges)
        bd, bends = refs.brute_force(labels, edges, q, v_s, j0, j1)
        d, ev, ej = O.dp_dense_at(g, q, v_s, j0, j1=j1)
        assert d == bd and (ev, ej) == min(bends), (case, labels, edges, q, v_s, j0, j1)
        gw = O.gwf(g, q, v_s, j0=j0, j1=j1)
        assert (gw["dist"], gw["end_v"], gw["end_j"]) == (d, ev, ej), case
        v_e = int(rng.integers(0, len(labels)))
        want = refs.brute_force_global(labels, edges, q, v_s, v_e, j0, j1)
        assert O.dp_dense_at(g, q, v_s, j0, v_e, j1=j1)[0] == want, (case, v_e)
        gg = O.gwf(g, q, v_s, v_e=v_e, j0=j0, j1=j1)
        assert (gg["dist"] if gg["status"] == 0 else -1) == want, case
    assert n_win > 100


def test_start_window_is_the_minimum_over_its_starts():
    rng = np.random.default_rng(772)
    for case in range(100):
        labels, edges, q, v_s = refs.random_case(rng, n_vtx=int(rng.integers(1, 6)), max_label=8,
                                                 p_edge=0.3, qlen=int(rng.integers(0, 12)))
        L = len(labels[v_s])
        j0 = int(rng.integers(0, L + 1))
        j1 = int(rng.integers(j0, L + 1))
        g = (labels, edges)
        d = O.dp_dense_at(g, q, v_s, j0, j1=j1)[0]
        assert d == min(O.dp_dense_at(g, q, v_s, j)[0] for j in range(j0, j1 + 1)), case


# ---------------------------------------------------------------------------
# a free end gap in the query: up to e trailing bases left unaligned
# ---------------------------------------------------------------------------
def test_query_end_gap_hand_cases():
    g = (["ACGT", "TT"], [(0, 1)])
    q = b"ACGTTGGG"
    # e = 0: ACGTT then three insertions, tied with a mismatch + two
    # insertions against ACGTTT; the smaller end cell wins
    assert O.dp_dense_clip(g, q, 0, 0) == (3, 1, 1, 0)
    # e = 2: row 6 (ACGTTG) costs 1 (an insertion after ACGTT)
    assert O.dp_dense_clip(g, q, 0, 2) == (1, 1, 1, 2)
    # e >= 3: ACGTT is spelled exactly; clipping more does not help and the
    # largest such row wins
    assert O.dp_dense_clip(g, q, 0, 3) == (0, 1, 1, 3) == O.dp_dense_clip(g, q, 0, 8)
    # global form, end vertex 1 (all of TT): ACGTTG against ACGTTT
    assert O.dp_dense_clip(g, q, 0, 2, v_e=1) == (1, 1, 2, 2)
    for e, want in ((0, 0), (2, 2), (3, 3), (8, 3)):
        assert O.gwf(g, q, 0, e=e)["clip"] == want


def test_query_end_gap_brute_force_random_tiny():
    rng = np.random.default_rng(881)
    n_clip = 0
    for case in range(300):
        labels, edges, q, v_s = refs.random_case(rng, n_vtx=int(rng.integers(1, 5)), max_label=4,
                                                 p_edge=0.35, qlen=int(rng.integers(0, 8)))
        e = int(rng.integers(0, len(q) + 1))
        L = len(labels[v_s])
        j0 = int(rng.integers(0, L + 1))
        j1 = int(rng.integers(j0, L + 1)) if rng.random() < 0.3 else j0
        g = (labels, edges)
        bd, bends, bclip = refs.brute_force_clip(labels, edges, q, v_s, e, j0, j1)
        d, ev, ej, clip = O.dp_dense_clip(g, q, v_s, e, j0, j1)
        n_clip += clip > 0
        assert (d, clip) == (bd, bclip) and (ev, ej) == min(bends), (case, labels, edges, q, v_s, e, j0, j1)
        gw = O.gwf(g, q, v_s, j0=j0, j1=j1, e=e)
        assert (gw["dist"], gw["end_v"], gw["end_j"], gw["clip"]) == (d, ev, ej, clip), case
        v_e = int(rng.integers(0, len(labels)))
        wd, wclip = refs.brute_force_global_clip(labels, edges, q, v_s, v_e, e, j0, j1)
        dg, _, _, cg = O.dp_dense_clip(g, q, v_s, e, j0, j1, v_e)
        assert (dg, cg if dg >= 0 else 0) == (wd, wclip), (case, v_e)
        gg = O.gwf(g, q, v_s, v_e=v_e, j0=j0, j1=j1, e=e)
        assert ((gg["dist"], gg["clip"]) if gg["status"] == 0 else (-1, 0)) == (wd, wclip), case
    assert n_clip > 50


def test_query_end_gap_zero_is_the_plain_form_and_full_gap_is_the_longest_spelled_prefix():
    rng = np.random.default_rng(882)
    for case in range(100):
        labels, edges, q, v_s = refs.random_case(rng, n_vtx=int(rng.integers(1, 6)), max_label=6,
                                                 p_edge=0.3, qlen=int(rng.integers(0, 14)))
        g = (labels, edges)
        assert O.dp_dense_clip(g, q, v_s, 0)[:3] == O.dp_dense_at(g, q, v_s), case
        # clipping everything: distance 0, keeping the longest prefix of q
        # that some walk from the start spells exactly
        d, _, _, clip = O.dp_dense_clip(g, q, v_s, len(q))
        longest = max(i for i in range(len(q) + 1) if O.dp_dense_at(g, q[:i], v_s)[0] == 0)
        assert (d, clip) == (0, len(q) - longest), case


# ---------------------------------------------------------------------------
# global form with a free end gap in the walk: the walk may end anywhere
# inside v_e (one of the variants Section 2.2 points to)
# ---------------------------------------------------------------------------
def test_walk_end_gap_hand_cases():
    g = (["ACGT", "TTGCA"], [(0, 1)])
    # ACGTTTG: ends after TTG (the CA left unspelled is free)
    assert O.dp_dense_at(g, b"ACGTTTG", 0, v_e=1, wfree=True) == (0, 1, 3)
    assert O.gwf(g, b"ACGTTTG", 0, v_e=1, wfree=True)["end_j"] == 3
    # the fixed end pays for the two unspelled bases
    assert O.dp_dense_at(g, b"ACGTTTG", 0, v_e=1)[0] == 2
    # ACGTTG: ACGTT plus an insertion, tied with ACGTTT and a mismatch; the
    # smaller end offset wins
    assert O.dp_dense_at(g, b"ACGTTG", 0, v_e=1, wfree=True) == (1, 1, 1)
    # ACGT: the walk must enter v_e; one base of it costs one deletion
    assert O.dp_dense_at(g, b"ACGT", 0, v_e=1, wfree=True) == (1, 1, 1)
    # ending inside the start vertex: ACG is spelled by v_0 alone
    assert O.dp_dense_at(g, b"ACG", 0, v_e=0, wfree=True) == (0, 0, 3)
    # empty query, v_e = v_s, offset 0: the start cell itself ends the walk
    assert O.dp_dense_at(g, b"", 0, v_e=0, wfree=True) == (0, 0, 0)
    # with a start offset the start cell (v_s, 2) is an ordinary end cell
    assert O.dp_dense_at(g, b"", 0, 2, v_e=0, wfree=True) == (0, 0, 2)
    assert O.dp_dense_at(g, b"", 0, v_e=1, wfree=True) == (5, 1, 1)


def test_walk_end_gap_brute_force_random_tiny():
    """The dense form and Algorithms 1-3 against walk enumeration (every walk
    to v_e cut after every base of v_e), with start offsets and windows, and
    with a free end gap in the query against enumeration over its prefixes."""
    rng = np.random.default_rng(991)
    n_inside = 0
    for case in range(300):
        labels, edges, q, v_s = refs.random_case(rng, n_vtx=int(rng.integers(1, 5)), max_label=5,
                                                 p_edge=0.35, qlen=int(rng.integers(0, 8)))
        L = len(labels[v_s])
        j0 = int(rng.integers(0, L + 1)) if rng.random() < 0.5 else 0
        j1 = int(rng.integers(j0, L + 1)) if rng.random() < 0.3 else j0
        v_e = int(rng.integers(0, len(labels)))
        g = (labels, edges)
        bd, bends = refs.brute_force_global_wfree(labels, edges, q, v_s, v_e, j0, j1)
        d, ev, ej = O.dp_dense_at(g, q, v_s, j0, v_e, j1=j1, wfree=True)
        if bd < 0:
            assert d == -1, case
            assert O.gwf(g, q, v_s, v_e=v_e, j0=j0, j1=j1, wfree=True)["status"] == 2, case
            continue
        assert (d, ev, ej) == (bd, v_e, min(bends)), (case, labels, edges, q, v_s, v_e, j0, j1)
        n_inside += ej < len(labels[v_e])
        gw = O.gwf(g, q, v_s, v_e=v_e, j0=j0, j1=j1, wfree=True)
        assert (gw["status"], gw["dist"], gw["end_v"], gw["end_j"]) == (0, d, ev, ej), case
        # never worse than the fixed end, which is one of its candidates
        fixed = O.dp_dense_at(g, q, v_s, j0, v_e, j1=j1)[0]
        assert d <= fixed, case
        # with a free end gap in the query: the best over prefixes, ties to the longest
        e = int(rng.integers(0, len(q) + 1))
        want = min((refs.brute_force_global_wfree(labels, edges, q[:i], v_s, v_e, j0, j1)[0], -i)
                   for i in range(len(q) - e, len(q) + 1))
        dc, _, _, clip = O.dp_dense_clip(g, q, v_s, e, j0, j1, v_e, wfree=True)
        assert (dc, -(len(q) - clip)) == want, (case, e)
        gc = O.gwf(g, q, v_s, v_e=v_e, j0=j0, j1=j1, e=e, wfree=True)
        assert (gc["dist"], gc["clip"]) == (dc, clip), (case, e)
    assert n_inside > 50


def test_walk_end_gap_on_chains_is_the_best_prefix_ending_in_the_end_vertex():
    """On a chain the free walk end is the textbook edit distance of the
    query against the best prefix of the spelled chain that ends inside v_e."""
    rng = np.random.default_rng(992)
    for case in range(80):
        nv = int(rng.integers(1, 7))
        labels = ["".join("ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(1, 6)))) for _ in range(nv)]
        edges = [(i, i + 1) for i in range(nv - 1)]
        a = int(rng.integers(0, nv))
        b = int(rng.integers(a, nv))
        q = "".join("ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(0, 14)))).encode()
        before = len("".join(labels[a:b]))
        t = "".join(labels[a:b + 1]).encode()
        lo = 0 if (a == b) else before + 1
        want = min(refs.ed(q, t[:p]) for p in range(lo, len(t) + 1))
        assert O.dp_dense_at((labels, edges), q, a, v_e=b, wfree=True)[0] == want, case
        assert O.gwf((labels, edges), q, a, v_e=b, wfree=True)["dist"] == want, case


# ---------------------------------------------------------------------------
# Algorithm 4 and the walk length W~ (reading R12), pinned on graphs where
# every walk from the start has the same length up to each base: chains and
# SNP bubbles.  There W~ of a front cell is its walk position, and the
# graph transcription with pruning must agree with an independent pairwise
# wavefront that applies the same keep rule to a = i + j.
# ---------------------------------------------------------------------------
def test_pairwise_pruned_reference_is_pinned():
    """The pairwise reference itself: without pruning it is the textbook
    extension-form edit distance (best over prefixes of the text, ending
    position the shortest such prefix); with pruning never below it."""
    rng = np.random.default_rng(4101)
    for _ in range(300):
        t = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, size=int(rng.integers(1, 60)))].tobytes()
        q = refs.mutate(rng, t[:int(rng.integers(0, len(t) + 1))], float(rng.uniform(0, 0.3)))
        cols = [frozenset([c]) for c in t]
        row = refs.semiglobal_ed_row(q, t)
        d, j = refs.pairwise_wf_pruned(q, cols)
        assert d == int(row.min()) and j == int(np.argmin(row)), (q, t)
        for a in (2, 5, 11):
            assert refs.pairwise_wf_pruned(q, cols, a)[0] >= d


def _walk_pos(pos, v, j):
    return pos[v] + j


@pytest.mark.parametrize("kind", ["chain", "snp"])
def test_algorithm4_matches_pairwise_pruning(kind):
    """Distance and end position of orc_gwf with Algorithm 4 equal the
    pairwise wavefront with the same keep rule, at several a_diff, on
    queries with errors; every extended entry's W~ is its walk position."""
    rng = np.random.default_rng(4102 if kind == "chain" else 4103)
    n_pruned_differs = 0
    for case in range(250):
        length = int(rng.integers(20, 300))
        if kind == "chain":
            labels, edges, cols, pos = refs.chain_case(rng, length, int(rng.integers(1, 25)))
        else:
            labels, edges, cols, pos = refs.snp_bubble_case(rng, length, float(rng.uniform(0.05, 0.3)),
                                                            int(rng.integers(1, 12)))
        t = refs.spell_cols(rng, cols)
        q = refs.mutate(rng, t[:int(rng.integers(0, length + 1))], float(rng.uniform(0.0, 0.3)))
        exact = None
        for a_diff in (0, 1, 2, 3, 4, 6, 10, 17, 30, 80):
            ref = refs.pairwise_wf_pruned(q, cols, a_diff)
            got = O.gwf((labels, edges), q, 0, a_diff=a_diff, entries_cap=1 << 16)
            assert got["status"] == 0
            assert (got["dist"], _walk_pos(pos, got["end_v"], got["end_j"])) == ref, (case, a_diff, labels, q)
            if a_diff == 0:
                exact = got["dist"]
                assert exact == O.dp_dense((labels, edges), q, 0)[0]
            elif got["dist"] > exact:
                n_pruned_differs += 1
            ent = got["entries"]
            assert got["entries_total"] == len(ent) == got["work"]
            # W~ (reading R12) is the walk position of the front cell
            assert (ent[:, 4] == np.asarray(pos)[ent[:, 1]] + ent[:, 3]).all(), (case, a_diff)
    # the keep rule decided something: pruning changed some distances
    assert n_pruned_differs > 100


def test_walk_length_with_a_start_offset_on_chains():
    """With the walk starting after j0 bases of v_s, W~ counts walk bases
    from there: W~ = position - j0 on every entry of every score."""
    rng = np.random.default_rng(4104)
    for _ in range(150):
        labels, edges, cols, pos = refs.chain_case(rng, int(rng.integers(10, 200)), int(rng.integers(2, 30)))
        j0 = int(rng.integers(0, len(labels[0]) + 1))
        t = refs.spell_cols(rng, cols)[j0:]
        q = refs.mutate(rng, t[:int(rng.integers(0, len(t) + 1))], float(rng.uniform(0.0, 0.2)))
        for a_diff in (0, 5, 20):
            got = O.gwf((labels, edges), q, 0, a_diff=a_diff, j0=j0, entries_cap=1 << 16)
            ref = refs.pairwise_wf_pruned(q, cols[j0:], a_diff)
            assert (got["dist"], _walk_pos(pos, got["end_v"], got["end_j"]) - j0) == ref
            ent = got["entries"]
            assert (ent[:, 4] == np.asarray(pos)[ent[:, 1]] + ent[:, 3] - j0).all()


# ---------------------------------------------------------------------------
# The value-capped oracle is the reference of every full-size comparison, so
# it is pinned against the dense oracle on many graphs: 10,000 tiny random
# graphs (cycles, self-loops) and medium graphs with queries up to 3 kb.
# ---------------------------------------------------------------------------
def test_capped_equals_dense_10k_tiny_graphs():
    rng = np.random.default_rng(4201)
    n_cut = 0
    for _ in range(10000):
        labels, edges, q, vs = refs.random_case(rng, n_vtx=int(rng.integers(1, 9)), max_label=6,
                                                p_edge=float(rng.uniform(0.1, 0.5)), qlen=int(rng.integers(0, 40)))
        d, ev, ej, _ = O.dp_dense((labels, edges), q, vs)
        D = d + int(rng.integers(0, 4))
        assert O.dp_capped((labels, edges), q, vs, D) == (d, ev, ej), (labels, edges, q, vs, D)
        if d > 0:
            assert O.dp_capped((labels, edges), q, vs, d - 1)[0] == -1
            n_cut += 1
    assert n_cut > 8000


def test_capped_equals_dense_medium_graphs():
    """Medium graphs (20-200 vertices, labels up to 400 bases, bubbles, back
    edges, self-loops) with queries of 50-3,000 bases at 0-12% error:
    capped at the exact distance, and at a few values above it, the capped
    oracle gives the dense oracle's distance and end."""
    rng = np.random.default_rng(4202)
    big = 0
    for _ in range(200):
        labels, edges, q, vs, _ = refs.medium_case(rng)
        d, ev, ej, _ = O.dp_dense((labels, edges), q, vs)
        for D in (d, d + 7, 2 * d + 1):
            assert O.dp_capped((labels, edges), q, vs, D) == (d, ev, ej), (D, d)
        if d > 0:
            assert O.dp_capped((labels, edges), q, vs, d - 1)[0] == -1
        big += d >= 100
    assert big >= 30


# ---------------------------------------------------------------------------
# W~ where walks differ in length (indels, loops): soundness against Eq. 1
# with the walk length as an extra index, and the tie rules of the reading
# of W~ against an independent implementation of it.
# ---------------------------------------------------------------------------
def test_walk_length_is_a_real_walk_at_the_entry_score():
    """Every extended entry (s, v, k, off, W~) of orc_gwf has a walk of
    exactly W~ bases from the start to its front cell that aligns q[1..i]
    at cost <= s (the chain of expansions, extensions and crossings that
    made the entry costs exactly s); exact and pruned, with and without a
    start offset, on tiny random graphs with cycles and self-loops.  An
    insertion that advanced W~ (a planted slip, in the independent
    implementation below) fails this."""
    rng = np.random.default_rng(4301)
    n_checked = n_slip = 0
    for _ in range(200):
        labels, edges, q, vs = refs.random_case(rng, n_vtx=int(rng.integers(2, 7)), max_label=5,
                                                p_edge=float(rng.uniform(0.15, 0.5)), qlen=int(rng.integers(0, 25)))
        j0 = int(rng.integers(0, len(labels[vs]) + 1)) if rng.random() < 0.3 else 0
        C = pos = None
        for a_diff in (0, 3, 8):
            got = O.gwf((labels, edges), q, vs, a_diff=a_diff, j0=j0, entries_cap=1 << 16)
            ent = got["entries"]
            assert len(ent) == got["work"]
            w_need = int(ent[:, 4].max()) + 1
            if C is None or C.shape[1] < w_need + 1:
                C, pos = refs.walk_length_costs(labels, edges, q, vs, w_need + 8, j0)
            for s, v, k, o, W in ent.tolist():
                assert refs.front_cell_cost(C, pos, labels, edges, vs, j0, k + o, v, o, W) <= s, \
                    (labels, edges, q, vs, j0, a_diff, (s, v, k, o, W))
                n_checked += 1
            if j0 == 0:
                _, _, slip = refs.gwf_walk_lengths(labels, edges, q, vs, a_diff, variant="ins_w")
                if any(refs.front_cell_cost(C, pos, labels, edges, vs, 0, k + o, v, o, W) > s
                       for s, v, k, o, W in slip):
                    n_slip += 1
    assert n_checked > 20000
    assert n_slip > 100


def test_walk_length_tie_rules_match_an_independent_implementation():
    """orc_gwf's distance, end and every extended entry (score, v, k, off,
    W~) equal those of an independent implementation of Algorithms 1-4 with
    the same reading of W~ (the larger W~ on offset ties, crossings in rounds
    with the larger W~ within a round and an earlier round first), exact and
    at several a_diff, on tiny random graphs with cycles and self-loops and
    on medium graphs with indel bubbles.  Each plausible alternative rule
    (the smaller W~, the first crossing of a round, depth-first crossings
    without rounds, an insertion advancing W~) disagrees with the oracle on
    many of these runs, so the inputs exercise every rule."""
    rng = np.random.default_rng(4302)
    variants = ("min_w", "first_w", "lifo", "ins_w")
    differs = dict.fromkeys(variants, 0)
    runs = 0

    def check(labels, edges, q, vs, a_diff, j0=0):
        nonlocal runs
        got = O.gwf((labels, edges), q, vs, a_diff=a_diff, j0=j0, entries_cap=1 << 22)
        assert got["status"] == 0 and got["entries_total"] == len(got["entries"])
        mine = (got["dist"], (got["end_v"], got["end_j"]), sorted(map(tuple, got["entries"].tolist())))
        assert refs.gwf_walk_lengths(labels, edges, q, vs, a_diff, j0) == mine, (labels, edges, q, vs, a_diff, j0)
        for var in variants:
            differs[var] += refs.gwf_walk_lengths(labels, edges, q, vs, a_diff, j0, variant=var) != mine
        runs += 1

    for _ in range(300):
        labels, edges, q, vs = refs.random_case(rng, n_vtx=int(rng.integers(2, 8)), max_label=5,
                                                p_edge=float(rng.uniform(0.15, 0.5)), qlen=int(rng.integers(0, 30)))
        j0 = int(rng.integers(0, len(labels[vs]) + 1)) if rng.random() < 0.3 else 0
        for a_diff in (0, 2, 5, 12):
            check(labels, edges, q, vs, a_diff, j0)
    for _ in range(20):
        labels, edges, q, vs, _ = refs.medium_case(rng)
        q = q[:int(rng.integers(50, 800))]
        for a_diff in (0, 10, 40):
            check(labels, edges, q, vs, a_diff)
    assert runs == 1260
    assert min(differs.values()) > 100, differs
