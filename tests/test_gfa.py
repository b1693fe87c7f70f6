"""GFA 1 input (gwfa_gfa_*, host code): segments and oriented links become
the strand-doubled graph of Definition 2.1.  Pinned against a plain Python
reading of the records, the strand symmetry every such graph has, and the
oracle: a query spelled along an oriented segment path aligns at distance 0,
and so does its reverse complement along the reversed path."""
import numpy as np
import pytest

import oracle as O
from tests import refs

gw = pytest.importorskip("paper_2206_13574_amd.gwfa")


def _labels(g):
    return [g.label(v).decode() for v in range(g.n_vtx)]


def _edges(g):
    return sorted(zip(g.edge_src.tolist(), g.edge_dst.tolist()))


def test_hand_example():
    text = "H\tVN:Z:1.0\nS\ts1\tACG\nS\ts2\tTTA\nL\ts1\t+\ts2\t-\t0M\n"
    G = gw.GFA(text=text)
    assert _labels(G.graph) == ["ACG", "CGT", "TTA", "TAA"]
    assert _edges(G.graph) == [(0, 3), (2, 1)]      # s1+ -> s2-, and s2+ -> s1-
    assert G.vertex("s2", reverse=True) == 3 and G.name(3) == ("s2", True) and G.name(0) == ("s1", False)
    F = gw.GFA(text=text, forward_only=True)
    assert _labels(F.graph) == ["ACG", "TTA"] and _edges(F.graph) == [] and F.n_skipped == 1


@pytest.mark.parametrize("forward_only", [False, True])
def test_random_gfa_against_plain_reading(forward_only):
    rng = np.random.default_rng(11 + forward_only)
    for case in range(200):
        text = refs.random_gfa(rng, n_seg=int(rng.integers(1, 9)), n_links=int(rng.integers(0, 15)))
        if rng.random() < 0.3:
            text = text.replace("\n", "\r\n")
        G = gw.GFA(text=text, forward_only=forward_only)
        labels, edges, skipped = refs.gfa_reference(text.replace("\r", ""), forward_only)
        assert _labels(G.graph) == labels, case
        assert _edges(G.graph) == edges, case
        assert G.n_skipped == skipped


def test_strand_symmetry():
    rng = np.random.default_rng(5)
    for _ in range(100):
        G = gw.GFA(text=refs.random_gfa(rng)).graph
        lab = _labels(G)
        es = set(_edges(G))
        for v in range(0, G.n_vtx, 2):
            assert lab[v + 1] == refs.revcomp(lab[v])
        for u, w in es:
            assert (w ^ 1, u ^ 1) in es


def test_oriented_path_aligns_exactly_both_strands():
    """A query spelled along s_a^oa, s_b^ob, ... (linked in the file) has
    distance 0 from the vertex of its first oriented segment; its reverse
    complement has distance 0 from the complement of the last one."""
    rng = np.random.default_rng(9)
    n_ok = 0
    for case in range(150):
        text = refs.random_gfa(rng, n_seg=6, n_links=14, extras=False)
        G = gw.GFA(text=text)
        g = G.graph
        succ = {}
        for u, w in _edges(g):
            succ.setdefault(u, []).append(w)
        v = int(rng.integers(0, g.n_vtx))
        walk = [v]
        for _ in range(int(rng.integers(0, 5))):
            if not succ.get(walk[-1]):
                break
            walk.append(succ[walk[-1]][int(rng.integers(0, len(succ[walk[-1]])))])
        spelled = "".join(g.label(x).decode() for x in walk)
        d, _, _, _ = O.dp_dense(g, spelled.encode(), walk[0])
        assert d == 0, case
        rc = refs.revcomp(spelled)
        d2, _, _, _ = O.dp_dense(g, rc.encode(), walk[-1] ^ 1)
        assert d2 == 0, case
        # the names and orientations of the walk read back
        names = [G.name(x) for x in walk]
        assert [G.vertex(n, r) for n, r in names] == walk
        n_ok += len(walk) > 1
    assert n_ok > 50


@pytest.mark.parametrize("text,code,line", [
    ("S\ts1\tACGN\n", gw.ERR_ALPHABET, 1),
    ("S\ts1\t*\n", gw.ERR_UNSUPPORTED, 1),
    ("S\ts1\tAC\nS\ts1\tGT\n", gw.ERR_FORMAT, 2),
    ("S\ts1\tAC\nL\ts1\t+\ts2\t+\t0M\n", gw.ERR_VERTEX, 2),
    ("S\ts1\tAC\nL\ts1\t+\ts1\t+\t3M\n", gw.ERR_UNSUPPORTED, 2),
    ("S\ts1\tAC\nL\ts1\tx\ts1\t+\t0M\n", gw.ERR_FORMAT, 2),
    ("S\ts1\tAC\nL\ts1\t+\ts1\n", gw.ERR_FORMAT, 2),
    ("S\ts1\n", gw.ERR_FORMAT, 1),
    ("S\ts1\t\n", gw.ERR_EMPTY_LABEL, 1),
    ("H\tVN:Z:1.0\n", gw.ERR_FORMAT, 0),
])
def test_errors(text, code, line):
    with pytest.raises(gw.GwfaError) as e:
        gw.GFA(text=text)
    assert e.value.code == code
    assert (f"line {line}" in str(e.value)) == (line > 0)


def test_file_and_forward_vertex_lookup(tmp_path):
    p = tmp_path / "g.gfa"
    p.write_text("S\ta\tAC\nS\tb\tGT\nL\ta\t+\tb\t+\t*\nL\ta\t-\tb\t+\t0M\n")
    F = gw.GFA(str(p), forward_only=True)
    assert _edges(F.graph) == [(0, 1)] and F.n_skipped == 1 and F.vertex("b") == 1
    with pytest.raises(gw.GwfaError):
        F.vertex("b", reverse=True)
    with pytest.raises(gw.GwfaError) as e:
        gw.GFA(str(tmp_path / "missing.gfa"))
    assert e.value.code == gw.ERR_ARG
