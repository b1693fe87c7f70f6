"""The command-line aligner's host side (no GPU): FASTA/FASTQ reading and
oriented segment names."""
import pytest

from paper_2206_13574_amd import align

gw = pytest.importorskip("paper_2206_13574_amd.gwfa")


def test_fasta_and_fastq(tmp_path):
    fa = tmp_path / "r.fa"
    fa.write_text(">r1 some description\nACGT\nTT\n\n>r2\nGGA\n")
    assert align.read_queries(str(fa)) == (["r1", "r2"], ["ACGTTT", "GGA"])
    fq = tmp_path / "r.fq"
    fq.write_text("@q1\nACGT\n+\nIIII\n@q2 x\nTT\n+\nII\n")
    assert align.read_queries(str(fq)) == (["q1", "q2"], ["ACGT", "TT"])
    bad = tmp_path / "bad.txt"
    bad.write_text("ACGT\n")
    with pytest.raises(ValueError):
        align.read_queries(str(bad))


def test_oriented_names():
    G = gw.GFA(text="S\ts1\tACG\nS\ts2\tTT\nL\ts1\t+\ts2\t-\t0M\n")
    assert align.parse_oriented(G, "s2-") == 3 and align.parse_oriented(G, "s1+") == 0
    assert align.parse_oriented(G, "s1") == 0
    assert [align.oriented_name(G, v) for v in range(4)] == ["s1+", "s1-", "s2+", "s2-"]
