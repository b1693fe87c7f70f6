"""Seeded synthetic pan-genome-shaped graphs and reads.

This module only draws random inputs; it holds none of the alignment
arithmetic, and both the HIP path and the CPU oracle consume what it makes.

Graphs (Def. 2.1 of the paper: a directed graph whose vertices carry DNA
strings) are built along a uniform-random ACGT backbone with:

* SNP bubbles: the backbone base and one other base as two 1-base vertices;
* indel bubbles: an arm vertex plus a direct skip edge; half the arms are a
  backbone span (a deletion allele), half novel sequence (an insertion);
* structural bubbles: a backbone span in parallel with a novel alt arm;
* tandem-repeat loops: a backbone span cut into its own vertex with a
  self-edge, so walks may traverse it any number of times.

Event gaps are geometric with the configured mean, at least 2 bp, with at
least one backbone base between consecutive events; vertex ids follow the
backbone, so the graph is topologically ordered apart from self-loops.

Reads follow A19/A18 of the design notes: a forward walk from offset 0 of a
start vertex (uniform choice at branches, a configured number of laps at a
loop), L bases spelled, then per-base errors with probability e split evenly
among substitution (one of the three other bases), insertion (a random base
after the current one) and deletion.  The injected edit count is returned: it
bounds the read's distance from above.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)
# position of a byte in ACGT (as np.searchsorted(ACGT, byte)), by table
_CODE = np.searchsorted(ACGT, np.arange(256, dtype=np.uint8))


@dataclass
class Graph:
    seq: np.ndarray          # uint8 ASCII, labels concatenated
    seg_off: np.ndarray      # int64, n+1
    edge_src: np.ndarray     # int32
    edge_dst: np.ndarray     # int32
    pos: np.ndarray = None   # int64: backbone coordinate of each vertex (for read starts)
    meta: dict = field(default_factory=dict)

    @property
    def n_vtx(self) -> int:
        return int(len(self.seg_off) - 1)

    @property
    def n_edge(self) -> int:
        return int(len(self.edge_src))

    def label(self, v: int) -> bytes:
        return self.seq[self.seg_off[v]:self.seg_off[v + 1]].tobytes()

    @classmethod
    def from_labels(cls, labels, edges) -> "Graph":
        seq = np.frombuffer("".join(labels).encode(), dtype=np.uint8).copy()
        off = np.zeros(len(labels) + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(s) for s in labels])
        e = np.asarray(list(edges), dtype=np.int32).reshape(-1, 2)
        return cls(seq, off, np.ascontiguousarray(e[:, 0]), np.ascontiguousarray(e[:, 1]),
                   pos=np.arange(len(labels), dtype=np.int64))


@dataclass
class Reads:
    seq: np.ndarray          # uint8 ASCII, reads concatenated
    off: np.ndarray          # int64, n+1
    v_start: np.ndarray      # int32
    n_edits: np.ndarray      # int32 injected edits (upper bound on the distance)
    err_rate: np.ndarray     # float64 per-read error rate
    meta: dict = field(default_factory=dict)
    v_end: np.ndarray = None     # int32 last vertex of each generating walk (global-form end vertex)
    end_rest: np.ndarray = None  # int32 bases of v_end after the read's last spelled base

    @property
    def n(self) -> int:
        return int(len(self.v_start))

    def read(self, r: int) -> bytes:
        return self.seq[self.off[r]:self.off[r + 1]].tobytes()

    def subset(self, idx) -> "Reads":
        idx = np.asarray(idx, dtype=np.int64)
        lens = (self.off[1:] - self.off[:-1])[idx]
        off = np.zeros(len(idx) + 1, dtype=np.int64)
        off[1:] = np.cumsum(lens)
        seq = np.concatenate([self.seq[self.off[r]:self.off[r + 1]] for r in idx]) if len(idx) else \
            np.zeros(0, dtype=np.uint8)
        return Reads(seq, off, self.v_start[idx].copy(), self.n_edits[idx].copy(),
                     self.err_rate[idx].copy(), dict(self.meta),
                     None if self.v_end is None else self.v_end[idx].copy(),
                     None if self.end_rest is None else self.end_rest[idx].copy())


def _gaps(rng, mean, n_max, lo=2):
    p = 1.0 / max(float(mean), 1.0)
    return np.maximum(rng.geometric(p, size=n_max), lo)


def bubble_graph(seed: int, backbone_len: int, snp_gap=None, indel_gap=None, indel_arm=(1, 20),
                 sv_gap=None, sv_arm=(1000, 10000), loop_sites=0, loop_unit=(10, 200),
                 loop_jitter=0.2) -> Graph:
    rng = np.random.default_rng(seed)
    B = int(backbone_len)
    bb = ACGT[rng.integers(0, 4, size=B)]
    events = []   # (pos, kind, a, b)

    def schedule(mean, kind):
        if not mean:
            return
        n_max = int(B / max(mean, 1) * 1.5) + 16
        pos = np.cumsum(_gaps(rng, mean, n_max))
        pos = pos[pos < B - 2]
        for p in pos:
            events.append([int(p), kind, 0, 0])

    schedule(snp_gap, "snp")
    schedule(indel_gap, "indel")
    schedule(sv_gap, "sv")
    if loop_sites:
        spacing = B / (loop_sites + 1)
        for s in range(loop_sites):
            c = (s + 1) * spacing + rng.uniform(-loop_jitter, loop_jitter) * spacing
            events.append([int(c), "loop", 0, 0])
    events.sort(key=lambda e: (e[0], e[1]))

    labels, pos_of, edges = [], [], []

    def add(lab: np.ndarray, p: int) -> int:
        labels.append(lab)
        pos_of.append(p)
        return len(labels) - 1

    tails = []
    cur = 0

    def backbone_to(p):
        nonlocal cur, tails
        if p > cur:
            v = add(bb[cur:p], cur)
            for t in tails:
                edges.append((t, v))
            tails = [v]
            cur = p

    for p, kind, _, _ in events:
        if p < cur + 1:           # keep at least one backbone base between events
            continue
        if kind == "snp":
            if p + 1 >= B:
                continue
            backbone_to(p)
            ref = bb[p:p + 1]
            alt = ACGT[(int(np.searchsorted(ACGT, ref[0])) + int(rng.integers(1, 4))) % 4:][:1]
            a = add(ref.copy(), p)
            b = add(alt.copy(), p)
            for t in tails:
                edges.append((t, a))
                edges.append((t, b))
            tails = [a, b]
            cur = p + 1
        elif kind == "indel":
            ln = int(rng.integers(indel_arm[0], indel_arm[1] + 1))
            if rng.random() < 0.5:      # deletion allele: the arm is backbone
                if p + ln >= B:
                    continue
                backbone_to(p)
                a = add(bb[p:p + ln].copy(), p)
                cur = p + ln
            else:                       # insertion allele: novel arm
                backbone_to(p)
                a = add(ACGT[rng.integers(0, 4, size=ln)], p)
            for t in tails:
                edges.append((t, a))
            tails = tails + [a]
        elif kind == "sv":
            rl = int(rng.integers(sv_arm[0], sv_arm[1] + 1))
            al = int(rng.integers(sv_arm[0], sv_arm[1] + 1))
            if p + rl >= B:
                continue
            backbone_to(p)
            r_ = add(bb[p:p + rl].copy(), p)
            x_ = add(ACGT[rng.integers(0, 4, size=al)], p)
            for t in tails:
                edges.append((t, r_))
                edges.append((t, x_))
            tails = [r_, x_]
            cur = p + rl
        elif kind == "loop":
            ul = int(rng.integers(loop_unit[0], loop_unit[1] + 1))
            if p + ul >= B:
                continue
            backbone_to(p)
            u = add(bb[p:p + ul].copy(), p)
            for t in tails:
                edges.append((t, u))
            edges.append((u, u))
            tails = [u]
            cur = p + ul
    backbone_to(B)
    seq = np.concatenate(labels).astype(np.uint8)
    off = np.zeros(len(labels) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(x) for x in labels])
    e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    g = Graph(seq, off, np.ascontiguousarray(e[:, 0]), np.ascontiguousarray(e[:, 1]),
              pos=np.asarray(pos_of, dtype=np.int64))
    g.meta = dict(seed=seed, backbone_len=B, snp_gap=snp_gap, indel_gap=indel_gap, indel_arm=indel_arm,
                  sv_gap=sv_gap, sv_arm=sv_arm, loop_sites=loop_sites, loop_unit=loop_unit,
                  n_vtx=g.n_vtx, n_edge=g.n_edge, bases=int(off[-1]))
    return g


def _csr(g: Graph):
    n = g.n_vtx
    order = np.argsort(g.edge_src, kind="stable")
    dst = g.edge_dst[order]
    src = g.edge_src[order]
    cnt = np.bincount(src, minlength=n)
    o = np.zeros(n + 1, dtype=np.int64)
    o[1:] = np.cumsum(cnt)
    return o, dst


def sample_reads(g: Graph, seed: int, n_reads: int, length, err, laps=(1, 1),
                 chunk: int = 4096, max_tries: int = 64) -> Reads:
    """length: int, or callable(rng, n) -> int array.  err: float, or
    callable(rng, n) -> float array.  laps: (lo, hi) passes through a
    self-looped vertex."""
    rng = np.random.default_rng(seed)
    n = g.n_vtx
    lab_len = (g.seg_off[1:] - g.seg_off[:-1]).astype(np.int64)
    o, dst = _csr(g)
    src_sorted = np.repeat(np.arange(n), np.diff(o))
    selfloop = np.zeros(n, dtype=bool)
    selfloop[src_sorted[dst == src_sorted]] = True
    # successors other than the vertex itself, in CSR form
    keep = dst != src_sorted
    nd = dst[keep]
    ns = src_sorted[keep]
    ncnt = np.bincount(ns, minlength=n)
    no = np.zeros(n + 1, dtype=np.int64)
    no[1:] = np.cumsum(ncnt)

    if callable(length):
        L = np.asarray(length(rng, n_reads), dtype=np.int64)
    else:
        L = np.full(n_reads, int(length), dtype=np.int64)
    if callable(err):
        E = np.asarray(err(rng, n_reads), dtype=np.float64)
    else:
        E = np.full(n_reads, float(err), dtype=np.float64)

    starts = np.full(n_reads, -1, dtype=np.int64)
    walks = [None] * n_reads
    todo = np.arange(n_reads)
    for _ in range(max_tries):
        if len(todo) == 0:
            break
        m = len(todo)
        sv = rng.integers(0, n, size=m)
        cur = sv.copy()
        need = L[todo].copy()
        lap_left = np.zeros(m, dtype=np.int64)
        alive = np.ones(m, dtype=bool)
        segs_r, segs_v, segs_n = [], [], []
        first = np.ones(m, dtype=bool)
        # the walks still growing, in ascending order (as a mask over all m
        # would give them; the random draws below depend on that order)
        act = np.nonzero(need > 0)[0]
        while len(act):
            v = cur[act]
            # a self-looped vertex entered fresh gets its lap count
            fresh = selfloop[v] & (lap_left[act] == 0)
            if fresh.any():
                lap_left[act[fresh]] = rng.integers(laps[0], laps[1] + 1, size=int(fresh.sum()))
            take = np.minimum(lab_len[v], need[act])
            segs_r.append(act)
            segs_v.append(v)
            segs_n.append(take)
            need[act] -= take
            first[act] = False
            act2 = act[need[act] > 0]
            act = act2
            if len(act2) == 0:
                continue
            v2 = cur[act2]
            again = selfloop[v2] & (lap_left[act2] > 1)
            lap_left[act2[again]] -= 1
            mv = act2[~again]
            if len(mv):
                vv = cur[mv]
                lap_left[mv] = 0
                deg = no[vv + 1] - no[vv]
                dead = deg == 0
                alive[mv[dead]] = False
                if dead.any():
                    act = act[alive[act]]
                ok = mv[~dead]
                if len(ok):
                    pick = (rng.random(len(ok)) * deg[~dead]).astype(np.int64)
                    cur[ok] = nd[no[cur[ok]] + pick]
        good = alive & (need == 0)
        if segs_r:
            R = np.concatenate(segs_r)
            V = np.concatenate(segs_v)
            N = np.concatenate(segs_n)
            order = np.argsort(R, kind="stable")
            R, V, N = R[order], V[order], N[order]
            bounds = np.searchsorted(R, np.arange(m + 1))
            for li in np.nonzero(good)[0]:
                a, b = bounds[li], bounds[li + 1]
                walks[todo[li]] = (V[a:b], N[a:b])
        starts[todo[good]] = sv[good]
        todo = todo[~good]
    if len(todo):
        raise RuntimeError(f"could not place {len(todo)} reads of the requested length")

    # last vertex of each generating walk (the end vertex of a global-form
    # alignment of the read) and the bases of it the read does not spell
    v_end = np.array([int(walks[r][0][-1]) for r in range(n_reads)], dtype=np.int32)
    end_rest = np.array([int(lab_len[walks[r][0][-1]] - walks[r][1][-1]) for r in range(n_reads)], dtype=np.int32)

    # spell, then inject errors, in chunks of reads
    out_seqs, n_edits = [], np.zeros(n_reads, dtype=np.int32)
    for c0 in range(0, n_reads, chunk):
        c1 = min(n_reads, c0 + chunk)
        vs = np.concatenate([walks[r][0] for r in range(c0, c1)])
        ns_ = np.concatenate([walks[r][1] for r in range(c0, c1)])
        tot = int(ns_.sum())
        seg_start = np.repeat(g.seg_off[vs], ns_)
        within = np.arange(tot, dtype=np.int64) - np.repeat(np.cumsum(ns_) - ns_, ns_)
        clean = g.seq[seg_start + within]
        rl = L[c0:c1]
        rid = np.repeat(np.arange(c1 - c0), rl)
        u = rng.random(tot)
        kind = rng.integers(0, 3, size=tot)          # 0 sub, 1 ins, 2 del
        is_err = u < E[c0:c1][rid]
        sub = is_err & (kind == 0)
        ins = is_err & (kind == 1)
        dele = is_err & (kind == 2)
        codes = _CODE[clean]
        codes = np.where(sub, (codes + rng.integers(1, 4, size=tot)) % 4, codes)
        base = ACGT[codes]
        cnt = np.where(dele, 0, np.where(ins, 2, 1))
        outb = np.repeat(base, cnt)
        # the second copy of an inserted base is replaced by a random base
        pos_end = np.cumsum(cnt) - 1
        ins_pos = pos_end[ins]
        outb[ins_pos] = ACGT[rng.integers(0, 4, size=len(ins_pos))]
        out_rid = np.repeat(rid, cnt)
        n_edits[c0:c1] = np.bincount(rid[is_err], minlength=c1 - c0).astype(np.int32)
        lens = np.bincount(out_rid, minlength=c1 - c0)
        out_seqs.append((outb, lens))
    seq = np.concatenate([s for s, _ in out_seqs]).astype(np.uint8)
    lens = np.concatenate([ln for _, ln in out_seqs]).astype(np.int64)
    off = np.zeros(n_reads + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    return Reads(seq, off, starts.astype(np.int32), n_edits, E,
                 meta=dict(seed=seed, n_reads=n_reads, laps=laps), v_end=v_end, end_rest=end_rest)


# --------------------------------------------------------------------------
# Workloads (seeds fixed here)
# --------------------------------------------------------------------------
def cfg1():
    """5 kb backbone, SNP every ~100 bp, indel (1-20 bp arm) every ~500 bp;
    50 reads x 1 kb at 1% error."""
    g = bubble_graph(101, 5000, snp_gap=100, indel_gap=500, indel_arm=(1, 20))
    r = sample_reads(g, 102, 50, 1000, 0.01)
    return g, r


def cfg2(n_reads: int = 20000):
    """1 Mb backbone, SNP every ~1 kb, indel (1-50) every ~5 kb, structural
    bubble (1-10 kb arms) every ~100 kb; reads lognormal(median 10 kb,
    sigma 0.5) clipped to [1, 50] kb, per-read error U(0.1%, 5%)."""
    return cfg2_shaped(201, 202, n_reads)


def cfg2_shaped(graph_seed: int, read_seed: int, n_reads: int):
    """A graph and reads of cfg2's shape from other seeds (held-out sets)."""
    g = bubble_graph(graph_seed, 1_000_000, snp_gap=1000, indel_gap=5000, indel_arm=(1, 50),
                     sv_gap=100_000, sv_arm=(1000, 10000))

    def length(rng, n):
        return np.clip(np.round(rng.lognormal(np.log(1e4), 0.5, size=n)), 1000, 50000).astype(np.int64)

    def err(rng, n):
        return rng.uniform(0.001, 0.05, size=n)

    r = sample_reads(g, read_seed, n_reads, length, err)
    return g, r


def cfg3(n_reads: int = 2000, read_len: int = 100_000):
    """500 kb backbone with 200 tandem-repeat loops (unit 10-200 bp with a
    self-edge); reads of 100 kb passing each loop 1-30 times, 1% error."""
    g = bubble_graph(301, 500_000, loop_sites=200, loop_unit=(10, 200))
    r = sample_reads(g, 302, n_reads, read_len, 0.01, laps=(1, 30))
    return g, r


def cfg4(n_reads: int = 50000, sparse: bool = False):
    """10 Mb backbone at the cfg1 densities (or 10x sparser); reads
    U{10..30} kb at error U(1%, 10%)."""
    f = 10 if sparse else 1
    g = bubble_graph(401, 10_000_000, snp_gap=100 * f, indel_gap=500 * f, indel_arm=(1, 20))

    def length(rng, n):
        return rng.integers(10000, 30001, size=n)

    def err(rng, n):
        return rng.uniform(0.01, 0.10, size=n)

    r = sample_reads(g, 402, n_reads, length, err)
    return g, r


def small_random_graph(rng, n_vtx: int, max_label: int = 4, p_edge: float = 0.3, cyclic: bool = True):
    """Tiny random graph for brute-force checks: labels 1..max_label bases,
    random edges including self-loops and back edges when cyclic."""
    labels = ["".join("ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(1, max_label + 1))))
              for _ in range(n_vtx)]
    edges = []
    for a in range(n_vtx):
        for b in range(n_vtx):
            if not cyclic and b <= a:
                continue
            if rng.random() < p_edge:
                edges.append((a, b))
    return Graph.from_labels(labels, edges)
