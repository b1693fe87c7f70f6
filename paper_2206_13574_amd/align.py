"""Command-line aligner: queries from FASTA/FASTQ against a GFA 1 graph on
one GPU, through the library's device entry points.

Each query needs a start: an oriented segment (`name+` / `name-`), an
optional offset inside it and an optional end of a free start window, and
an optional end segment for the global form.  Give one start for every query
(--start) or one per query in a tab-separated file (--starts: query name,
start segment, then optionally offset, window end, end segment; '.' leaves a
field unset).  --query-end-free E lets up to E trailing query bases stay
unaligned at no cost (a soft clip); with end segments, --walk-end-free lets
the walk end anywhere inside its end segment.  Output, one tab-separated line per
query: name, length, status, distance, end segment, bases of it consumed,
start offset, query bases clipped, walk (oriented segment names), CIGAR of
the query against the walk's string.

Usage:
    python -m paper_2206_13574_amd.align --gfa graph.gfa --reads reads.fa --start s1+ [--cigar] [--out out.tsv]
"""
from __future__ import annotations

import argparse
import sys

import numpy as np

STATUS = {0: "OK", 1: "MAX_SCORE", 2: "ARENA", 3: "BAD_INPUT", 4: "UNREACHABLE"}


def read_queries(path: str):
    """(names, sequences) from FASTA or FASTQ text (first word of the header)."""
    names, seqs = [], []
    with open(path) as f:
        lines = [l.rstrip("\r\n") for l in f]
    i = 0
    while i < len(lines):
        l = lines[i]
        if not l:
            i += 1
            continue
        if l[0] == ">":
            names.append(l[1:].split()[0] if len(l) > 1 else f"q{len(names)}")
            parts = []
            i += 1
            while i < len(lines) and (not lines[i] or lines[i][0] != ">"):
                parts.append(lines[i].strip())
                i += 1
            seqs.append("".join(parts))
        elif l[0] == "@":
            names.append(l[1:].split()[0] if len(l) > 1 else f"q{len(names)}")
            seqs.append(lines[i + 1].strip())
            i += 4                                   # header, sequence, '+', qualities
        else:
            raise ValueError(f"{path}: line {i + 1} is neither a FASTA nor a FASTQ header")
    return names, seqs


def parse_oriented(gfa, spec: str) -> int:
    """Vertex of an oriented segment name ('s1+', 's1-'; no sign means +)."""
    if spec.endswith(("+", "-")):
        return gfa.vertex(spec[:-1], reverse=spec.endswith("-"))
    return gfa.vertex(spec)


def oriented_name(gfa, v: int) -> str:
    name, rev = gfa.name(int(v))
    return name + ("-" if rev else "+")


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gfa", required=True)
    ap.add_argument("--reads", required=True, help="FASTA or FASTQ")
    ap.add_argument("--start", help="oriented start segment for every query, e.g. s1+ (optionally :offset)")
    ap.add_argument("--starts", help="per-query starts: name, segment, [offset, window end, end segment]")
    ap.add_argument("--end", help="oriented end segment for every query (global form)")
    ap.add_argument("--prune", choices=("none", "heuristic", "learned"), default="none")
    ap.add_argument("--a-diff", type=int, default=50)
    ap.add_argument("--query-end-free", type=int, default=0,
                    help="trailing query bases that may stay unaligned at no cost")
    ap.add_argument("--walk-end-free", action="store_true",
                    help="with end segments: the walk may end anywhere inside its end segment")
    ap.add_argument("--cigar", action="store_true", help="also write CIGARs (base-level alignments)")
    ap.add_argument("--forward-only", action="store_true", help="one vertex per segment, + + links only")
    ap.add_argument("--out", default="-")
    a = ap.parse_args(argv)

    from . import gwfa
    gfa = gwfa.GFA(a.gfa, forward_only=a.forward_only)
    names, seqs = read_queries(a.reads)
    n = len(names)
    vs = np.zeros(n, np.int32)
    j0 = np.zeros(n, np.int32)
    j1 = np.full(n, -1, np.int32)
    ve = np.full(n, -1, np.int32)
    if a.starts:
        row = {}
        with open(a.starts) as f:
            for line in f:
                if line.strip() and not line.startswith("#"):
                    fld = line.rstrip("\r\n").split("\t")
                    row[fld[0]] = fld[1:]
        for i, nm in enumerate(names):
            if nm not in row:
                raise SystemExit(f"no start for query {nm}")
            fld = row[nm] + ["."] * 4
            vs[i] = parse_oriented(gfa, fld[0])
            j0[i] = int(fld[1]) if fld[1] != "." else 0
            j1[i] = int(fld[2]) if fld[2] != "." else -1
            ve[i] = parse_oriented(gfa, fld[3]) if fld[3] != "." else -1
    elif a.start:
        spec, _, off = a.start.partition(":")
        vs[:] = parse_oriented(gfa, spec)
        j0[:] = int(off) if off else 0
    else:
        raise SystemExit("give --start or --starts")
    if a.end:
        ve[:] = parse_oriented(gfa, a.end)
    j1 = np.where(j1 < 0, j0, j1).astype(np.int32)
    if (ve >= 0).any() and (ve < 0).any():
        raise SystemExit("either every query has an end segment or none has")

    if a.prune == "learned":
        from . import train_prune
        W = train_prune.load()
        o = gwfa.opts(prune=gwfa.PRUNE_LEARNED, keep_threshold=W["tau"], mlp_gate=W["gate"], mlp_period=W["period"],
                      query_end_free=a.query_end_free, walk_end_free=a.walk_end_free)
    elif a.prune == "heuristic":
        o = gwfa.opts(prune=gwfa.PRUNE_HEURISTIC, a_diff=a.a_diff, query_end_free=a.query_end_free,
                      walk_end_free=a.walk_end_free)
    else:
        o = gwfa.opts(query_end_free=a.query_end_free, walk_end_free=a.walk_end_free)

    ctx = gwfa.Context(0)
    graph = gwfa.Graph.of(ctx, gfa.graph)
    if a.prune == "learned":
        ctx.mlp_load(W["w_bf16"], W["scale"])
    seq = np.frombuffer("".join(seqs).encode(), dtype=np.uint8).copy()
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(s) for s in seqs])
    torch = ctx.torch
    batch = gwfa.upload_reads(ctx, seq, off, vs)
    out = gwfa.alloc_out(ctx, n, int(off[-1]) * 2 + 256 * n)

    def dev(x):
        return torch.from_numpy(np.ascontiguousarray(x, np.int32) if n else np.zeros(1, np.int32)).to(ctx.tdev)

    gwfa.step_dev(ctx, graph, batch, out, o, dev(ve) if (ve >= 0).any() else None, dev(j0), dev(j1))
    torch.cuda.synchronize(ctx.tdev)
    if int(out.err.cpu().item()) != 0:
        raise SystemExit("a query has a base outside ACGT")
    res, path, _ = gwfa.fetch(out, n)
    cig = None
    if a.cigar:
        cig = gwfa.cigar_dev(ctx, graph, batch, out)
    graph.close()
    ctx.close()

    fo = sys.stdout if a.out == "-" else open(a.out, "w")
    fo.write("#name\tlength\tstatus\tdist\tend\tend_off\tstart_off\tclip\twalk\tcigar\n")
    for i in range(n):
        r = res[i]
        walk = "."
        if r["path_off"] >= 0 and r["path_len"] > 0:
            walk = ",".join(oriented_name(gfa, v) for v in path[r["path_off"]:r["path_off"] + r["path_len"]])
        end = oriented_name(gfa, r["end_v"]) if r["status"] == 0 else "."
        cg = "."
        if cig is not None and cig[2][i] >= 0:
            ops, coff, clen = cig
            cg = gwfa.cigar_string(ops[coff[i]:coff[i] + clen[i]]) or "."
        fo.write(f"{names[i]}\t{len(seqs[i])}\t{STATUS.get(int(r['status']), r['status'])}\t{int(r['dist'])}\t"
                 f"{end}\t{int(r['end_off'])}\t{int(r['start_off'])}\t{int(r['clip'])}\t{walk}\t{cg}\n")
    if fo is not sys.stdout:
        fo.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
