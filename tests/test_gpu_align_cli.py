"""The command-line aligner end to end on the GPU: a GFA graph with an
inversion, queries from both strands in FASTA, per-query starts (with an
offset and a free window), one query with a tail that is not in the graph
and a free end gap in the query, distances against the oracle, walks and
CIGARs consistent with them."""
import numpy as np
import pytest

import oracle as O
from tests import refs

pytestmark = pytest.mark.gpu


def test_align_cli_on_gfa(gpu_lib, tmp_path):
    from paper_2206_13574_amd import align
    gw = gpu_lib
    rng = np.random.default_rng(31)
    segs = ["".join("ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(20, 60)))) for _ in range(8)]
    gfa = ["S\ts%d\t%s" % (i, s) for i, s in enumerate(segs)]
    gfa += ["L\ts%d\t+\ts%d\t+\t0M" % (i, i + 1) for i in range(7)]
    gfa += ["L\ts2\t+\ts5\t-\t0M", "L\ts5\t-\ts6\t+\t*"]            # an inversion arm
    (tmp_path / "g.gfa").write_text("\n".join(gfa) + "\n")
    G = gw.GFA(str(tmp_path / "g.gfa"))
    g = G.graph
    walks = [["s0+", "s1+", "s2+", "s3+"], ["s1+", "s2+", "s5-", "s6+"], ["s3-", "s2-", "s1-", "s0-"]]
    reads, starts = [], []
    for w_i, w in enumerate(walks):
        s = "".join(g.label(align.parse_oriented(G, x)).decode() for x in w)
        for rep in range(3):
            q = list(s[:int(rng.integers(30, len(s)))])
            for _ in range(rep):                                   # 0-2 substitutions
                p = int(rng.integers(0, len(q)))
                q[p] = "ACGT"[("ACGT".index(q[p]) + 1) % 4]
            name = f"w{w_i}_{rep}"
            reads.append((name, "".join(q)))
            starts.append((name, w[0]))
    # one query seeded inside its start segment, one with a free window
    s0 = g.label(align.parse_oriented(G, "s0+")).decode()
    reads.append(("inside", s0[7:] + segs[1][:20]))
    starts.append(("inside", "s0+", "7"))
    reads.append(("window", s0[11:] + segs[1][:25]))
    starts.append(("window", "s0+", "0", str(len(s0))))
    reads.append(("tail", segs[3] + segs[4][:15] + "".join("ACGT"[x] for x in rng.integers(0, 4, size=10))))
    starts.append(("tail", "s3+"))
    e = 12
    (tmp_path / "r.fa").write_text("".join(f">{n}\n{q}\n" for n, q in reads))
    (tmp_path / "s.tsv").write_text("".join("\t".join(x) + "\n" for x in starts))
    out = tmp_path / "out.tsv"
    assert align.main(["--gfa", str(tmp_path / "g.gfa"), "--reads", str(tmp_path / "r.fa"), "--starts",
                       str(tmp_path / "s.tsv"), "--cigar", "--query-end-free", str(e), "--out", str(out)]) == 0
    rows = [l.split("\t") for l in out.read_text().splitlines() if not l.startswith("#")]
    assert len(rows) == len(reads)
    for (name, q), st, row in zip(reads, starts, rows):
        assert row[0] == name and row[2] == "OK"
        v0 = align.parse_oriented(G, st[1])
        j0 = int(st[2]) if len(st) > 2 else 0
        j1 = int(st[3]) if len(st) > 3 else -1
        d, ev, ej, clip = O.dp_dense_clip(g, q.encode(), v0, min(e, len(q)), j0, j1=j1)
        assert (int(row[3]), align.parse_oriented(G, row[4]), int(row[5]), int(row[7])) == (d, ev, ej, clip), name
        if name == "tail":
            assert d == 0 and clip >= 1
        walk = [align.parse_oriented(G, x) for x in row[8].split(",")]
        assert walk[0] == v0 and O.is_walk(g, walk)
        so = int(row[6])
        T = O.spell_walk(g, walk, ej)[so:]
        assert O.ed_global(q.encode()[:len(q) - clip], T) == d
        assert refs.cigar_cost(q.encode(), T, [_op(x) for x in _split_cigar(row[9])]) == d


def _split_cigar(s):
    import re
    return [] if s.strip() == "." else re.findall(r"\d+[=XIDS]", s.strip())


def _op(tok):
    code = {"=": 7, "X": 8, "I": 1, "D": 2, "S": 4}[tok[-1]]
    return (int(tok[:-1]) << 4) | code
