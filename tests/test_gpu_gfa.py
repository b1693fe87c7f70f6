"""GPU parity on a graph read from GFA (both strands, inversion links):
distances and ends bit-exact against the dense oracle, walks re-scored."""
import numpy as np
import pytest

import oracle as O
from tests import refs
from tests.test_gpu_parity import reads_of

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-gfa] {msg}", flush=True)


def _random_gfa_text(rng, n_seg=120):
    segs = ["".join("ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(5, 40)))) for _ in range(n_seg)]
    recs = [f"S\ts{i}\t{s}" for i, s in enumerate(segs)]
    for i in range(n_seg - 1):               # a backbone, with branches and inversions
        recs.append(f"L\ts{i}\t+\ts{i + 1}\t+\t0M")
        if rng.random() < 0.3:
            j = int(rng.integers(0, n_seg))
            recs.append(f"L\ts{i}\t{'+-'[int(rng.integers(0, 2))]}\ts{j}\t{'+-'[int(rng.integers(0, 2))]}\t*")
    return "\n".join(recs) + "\n"


def test_gfa_graph_reads_on_both_strands(gpu_lib, tmp_path):
    gw = gpu_lib
    rng = np.random.default_rng(2468)
    p = tmp_path / "g.gfa"
    p.write_text(_random_gfa_text(rng))
    G = gw.GFA(str(p))
    g = G.graph
    succ = {}
    for u, w in zip(g.edge_src.tolist(), g.edge_dst.tolist()):
        succ.setdefault(u, []).append(w)
    qs, vs = [], []
    for _ in range(300):
        v = int(rng.integers(0, g.n_vtx))
        walk, s = [v], g.label(v).decode()
        while len(s) < 120 and succ.get(walk[-1]):
            walk.append(succ[walk[-1]][int(rng.integers(0, len(succ[walk[-1]])))])
            s += g.label(walk[-1]).decode()
        s = list(s[:int(rng.integers(1, 121))])
        for _ in range(int(rng.integers(0, 4))):      # a few edits
            i = int(rng.integers(0, len(s)))
            s[i] = "ACGT"[int(rng.integers(0, 4))]
        qs.append("".join(s).encode())
        vs.append(v)
    say(f"{g.n_vtx} vertices, {g.n_edge} edges, {len(qs)} reads")
    ctx = gw.Context(0)
    graph = gw.Graph.of(ctx, g)
    try:
        seq, off = reads_of(qs)
        res, paths = gw.align(ctx, graph, seq, off, np.asarray(vs, np.int32))
    finally:
        graph.close()
        ctx.close()
    for i, q in enumerate(qs):
        d, ev, ej, _ = O.dp_dense(g, q, vs[i])
        assert (res[i]["status"], res[i]["dist"], res[i]["end_v"], res[i]["end_off"]) == (0, d, ev, ej), i
        walk = [int(x) for x in paths[i]]
        assert walk[0] == vs[i] and O.is_walk(g, walk)
        assert O.ed_global(q, O.spell_walk(g, walk, ej)) == d
