"""Independent references used to pin the oracle (tests only).

Nothing here shares code with ``oracle/``: the edit distances are textbook
dynamic programs written out in numpy/Python, and the brute force enumerates
walks explicitly.
"""
from __future__ import annotations

import numpy as np


def ed(a: bytes, b: bytes) -> int:
    """Textbook global edit distance (unit costs)."""
    a = a.upper()
    b = b.upper()
    prev = list(range(len(b) + 1))
    for i in range(1, len(a) + 1):
        cur = [i] + [0] * len(b)
        for j in range(1, len(b) + 1):
            cur[j] = min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (a[i - 1] != b[j - 1]))
        prev = cur
    return prev[-1]


def semiglobal_ed_row(q: bytes, t: bytes) -> np.ndarray:
    """Returns D[p] = ed(q, t[:p]) for every prefix length p of t (query
    consumed globally, end free in t)."""
    q = np.frombuffer(q.upper(), dtype=np.uint8)
    t = np.frombuffer(t.upper(), dtype=np.uint8)
    n, m = len(q), len(t)
    # rows over t positions, columns over q positions: col[i] = ed(q[:i], t[:p])
    col = np.arange(n + 1, dtype=np.int64)
    out = np.empty(m + 1, dtype=np.int64)
    out[0] = col[n]
    for p in range(1, m + 1):
        new = np.empty_like(col)
        new[0] = p
        sub = col[:-1] + (q != t[p - 1])
        dele = col[1:] + 1
        best = np.minimum(sub, dele)
        for i in range(1, n + 1):
            x = best[i - 1]
            y = new[i - 1] + 1
            new[i] = x if x < y else y
        col = new
        out[p] = col[n]
    return out


def brute_force(labels, edges, q: bytes, v_s: int, j0: int = 0, j1: int = None):
    """Enumerates every walk from (v_s, j) for every start j in j0..j1
    (after the first j bases of v_s; j1 = None: j0 only) and every end
    position on its last vertex, with an edit-distance column carried along
    the spelled string; a branch is abandoned once its column minimum
    exceeds the best distance found (the column minimum never decreases as
    the string grows).  Returns (d*, end set {(v, j)})."""
    if j1 is None:
        j1 = j0
    q = (q.decode() if isinstance(q, (bytes, bytearray)) else q).upper()
    n = len(q)
    succ = {}
    for a, b in edges:
        succ.setdefault(a, []).append(b)
    best = [n]                  # the empty prefix: all insertions
    ends = {(v_s, j) for j in range(j0, j1 + 1)}   # dropped below as soon as something beats n
    qa = list(q)

    def step(col, c):
        new = [col[0] + 1]
        for i in range(1, n + 1):
            new.append(min(col[i - 1] + (qa[i - 1] != c), col[i] + 1, new[i - 1] + 1))
        return new

    limit = 2 * n + 1

    def dfs(v, col, depth, first=0):
        lab = labels[v].upper()
        for j in range(first, len(lab)):
            col = step(col, lab[j])
            depth += 1
            d = col[n]
            if d < best[0]:
                best[0] = d
                ends.clear()        # includes the empty-prefix start cell
            if d == best[0]:
                ends.add((v, j + 1))
                # the cell before v_s's first base also holds this value when
                # the walk can step from here into v_s (zero-cost carry); it
                # is an end cell only when the walk starts there
                if j + 1 == len(lab) and j0 == 0 and v_s in succ.get(v, []):
                    ends.add((v_s, 0))
            if min(col) > best[0] or depth > limit:
                return
        for u in succ.get(v, []):
            dfs(u, col, depth)

    for j in range(j0, j1 + 1):
        dfs(v_s, list(range(n + 1)), 0, j)
    return best[0], ends


def char_split(labels, edges):
    """Splits every vertex into a chain of one-base vertices (the paper's
    string/char-labelled equivalence).  Returns (labels, edges, first, last,
    cell_map) where cell_map[(v, j)] -> (v', j') for j >= 1."""
    nl, first, last, cmap = [], [], [], {}
    for v, s in enumerate(labels):
        first.append(len(nl))
        for j, ch in enumerate(s):
            cmap[(v, j + 1)] = (len(nl), 1)
            nl.append(ch)
        last.append(len(nl) - 1)
    ne = []
    for v, s in enumerate(labels):
        for j in range(len(s) - 1):
            ne.append((first[v] + j, first[v] + j + 1))
    for a, b in edges:
        ne.append((last[a], first[b]))
    return nl, ne, first, last, cmap


def random_case(rng, n_vtx=5, max_label=3, p_edge=0.3, qlen=None, cyclic=True):
    labels = ["".join("ACGT"[x] for x in rng.integers(0, 4, size=int(rng.integers(1, max_label + 1))))
              for _ in range(n_vtx)]
    edges = [(a, b) for a in range(n_vtx) for b in range(n_vtx)
             if (cyclic or b > a) and rng.random() < p_edge]
    if qlen is None:
        qlen = int(rng.integers(0, 9))
    q = "".join("ACGT"[x] for x in rng.integers(0, 4, size=qlen)).encode()
    v_s = int(rng.integers(0, n_vtx))
    return labels, edges, q, v_s


def spell_random_walk(rng, labels, edges, v_s, max_len):
    succ = {}
    for a, b in edges:
        succ.setdefault(a, []).append(b)
    out, v = [], v_s
    walk = [v_s]
    total = 0
    while True:
        s = labels[v]
        take = min(len(s), max_len - total)
        out.append(s[:take])
        total += take
        if total >= max_len or take < len(s) or not succ.get(v):
            break
        v = succ[v][int(rng.integers(0, len(succ[v])))]
        walk.append(v)
    return "".join(out).encode(), walk


def brute_force_global(labels, edges, q: bytes, v_s: int, v_e: int, j0: int = 0, j1: int = None) -> int:
    """The minimum of the single-start form over the starts j0..j1."""
    if j1 is not None and j1 > j0:
        vals = [brute_force_global(labels, edges, q, v_s, v_e, j) for j in range(j0, j1 + 1)]
        vals = [x for x in vals if x >= 0]
        return min(vals) if vals else -1
    return _brute_force_global(labels, edges, q, v_s, v_e, j0)


def _brute_force_global(labels, edges, q: bytes, v_s: int, v_e: int, j0: int = 0) -> int:
    """Global form with an end vertex: min over every walk from v_s (after
    its first j0 bases) to v_e of the edit distance between q and the walk's
    whole spelled string; -1 when v_e cannot be reached.  Walks longer than |q| + max(|q|, |S|) bases, S the
    shortest walk, cannot be optimal (their cost exceeds S's), which bounds
    the enumeration on cyclic graphs."""
    import heapq
    q = (q.decode() if isinstance(q, (bytes, bytearray)) else q).upper()
    n = len(q)
    succ = {}
    for a, b in edges:
        succ.setdefault(a, []).append(b)
    # shortest spelled length of a walk v_s ... v_e (whole labels)
    dist = {v_s: len(labels[v_s]) - j0}
    pq = [(len(labels[v_s]) - j0, v_s)]
    while pq:
        d, v = heapq.heappop(pq)
        if d > dist.get(v, 1 << 60):
            continue
        for u in succ.get(v, []):
            nd = d + len(labels[u])
            if nd < dist.get(u, 1 << 60):
                dist[u] = nd
                heapq.heappush(pq, (nd, u))
    if v_e not in dist:
        return -1
    limit = n + max(n, dist[v_e])
    best = [1 << 60]
    qa = list(q)

    def step(col, c):
        new = [col[0] + 1]
        for i in range(1, n + 1):
            new.append(min(col[i - 1] + (qa[i - 1] != c), col[i] + 1, new[i - 1] + 1))
        return new

    def dfs(v, col, depth, first=0):
        for ch in labels[v].upper()[first:]:
            col = step(col, ch)
            depth += 1
            if depth > limit or min(col) >= best[0]:
                return
        if v == v_e and col[n] < best[0]:
            best[0] = col[n]
        for u in succ.get(v, []):
            dfs(u, col, depth)

    dfs(v_s, list(range(n + 1)), 0, j0)
    return best[0]


CIGAR_OPS = {7: "=", 8: "X", 1: "I", 2: "D", 4: "S"}


def cigar_cost(q: bytes, t: bytes, ops) -> int:
    """Checks that CIGAR words (length << 4 | op) align q to t exactly (every
    '=' pairs equal bases, every 'X' unequal ones, all of both strings
    consumed) and returns the alignment's cost X + I + D.  A soft clip 'S'
    (query bases left unaligned) may only come last and costs nothing."""
    q, t = q.upper(), t.upper()
    i = j = cost = 0
    ops = list(ops)
    for x, w in enumerate(ops):
        n, op = int(w) >> 4, CIGAR_OPS[int(w) & 15]
        assert n > 0
        if op == "S":
            assert x == len(ops) - 1
            i += n
        elif op == "=":
            assert q[i:i + n] == t[j:j + n]
            i += n; j += n
        elif op == "X":
            assert all(q[i + x] != t[j + x] for x in range(n))
            i += n; j += n; cost += n
        elif op == "I":
            i += n; cost += n
        else:
            j += n; cost += n
    assert i == len(q) and j == len(t)
    return cost


_RC = str.maketrans("ACGTacgt", "TGCAtgca")


def revcomp(s: str) -> str:
    return s.translate(_RC)[::-1]


def gfa_reference(text: str, forward_only: bool = False):
    """Plain reading of GFA 1 S and L records (independent of the library's
    parser): returns (labels, sorted unique edges, skipped links).  Segment i
    is vertex 2i and its reverse complement 2i+1 (vertex i with
    forward_only); a link a oa b ob gives a^oa -> b^ob and b^-ob -> a^-oa."""
    names, seqs = {}, []
    lines = [l.rstrip("\r") for l in text.split("\n")]
    for l in lines:
        f = l.split("\t")
        if f[0] == "S":
            names[f[1]] = len(seqs)
            seqs.append(f[2])
    edges, skipped = set(), 0
    for l in lines:
        f = l.split("\t")
        if f[0] != "L":
            continue
        a, oa, b, ob = names[f[1]], f[2] == "-", names[f[3]], f[4] == "-"
        if forward_only:
            if oa or ob:
                skipped += 1
            else:
                edges.add((a, b))
            continue
        u, w = 2 * a + oa, 2 * b + ob
        edges.add((u, w))
        edges.add((w ^ 1, u ^ 1))
    if forward_only:
        labels = list(seqs)
    else:
        labels = [x for s in seqs for x in (s, revcomp(s))]
    return labels, sorted(edges), skipped


def random_gfa(rng, n_seg=8, max_len=6, n_links=12, extras=True):
    """Random GFA 1 text: segments, links with random orientations (self
    links and repeats included), other record types mixed in, lines in a
    shuffled order (links may come before their segments)."""
    segs = ["".join("ACGTacgt"[x] for x in rng.integers(0, 8, size=int(rng.integers(1, max_len + 1))))
            for _ in range(n_seg)]
    recs = [f"S\ts{i}\t{s}\tLN:i:{len(s)}" for i, s in enumerate(segs)]
    for _ in range(n_links):
        a, b = rng.integers(0, n_seg, size=2)
        oa, ob = "+-"[int(rng.integers(0, 2))], "+-"[int(rng.integers(0, 2))]
        ov = ["0M", "*"][int(rng.integers(0, 2))]
        recs.append(f"L\ts{a}\t{oa}\ts{b}\t{ob}\t{ov}")
    if extras:
        recs += ["P\tp1\ts0+,s1-\t*", "# comment", "W\tsample\t1\tchr1\t0\t5\t>s0<s1"]
    order = rng.permutation(len(recs))
    body = "\n".join(recs[i] for i in order)
    return "H\tVN:Z:1.0\n" + body + ("\n" if rng.random() < 0.5 else "")


def brute_force_clip(labels, edges, q: bytes, v_s: int, e: int, j0: int = 0, j1: int = None):
    """A free end gap of up to e query bases: walk enumeration for every
    query prefix q[:i], i >= |q| - e.  Returns (d*, end set of the largest i
    reaching d*, |q| - that i)."""
    best = None
    for i in range(len(q), len(q) - e - 1, -1):
        d, ends = brute_force(labels, edges, q[:i], v_s, j0, j1)
        if best is None or d < best[0]:
            best = (d, ends, len(q) - i)
    return best


def brute_force_global_clip(labels, edges, q: bytes, v_s: int, v_e: int, e: int, j0: int = 0, j1: int = None):
    """Global form with a free end gap: (d, clip), (-1, 0) when unreachable."""
    best = (-1, 0)
    for i in range(len(q), len(q) - e - 1, -1):
        d = brute_force_global(labels, edges, q[:i], v_s, v_e, j0, j1)
        if d >= 0 and (best[0] < 0 or d < best[0]):
            best = (d, len(q) - i)
    return best


def brute_force_global_wfree(labels, edges, q: bytes, v_s: int, v_e: int, j0: int = 0, j1: int = None):
    """Global form with a free end gap in the walk: every walk from v_s
    (after its first j bases, j0 <= j <= j1) that reaches v_e, cut after any
    j >= 1 bases of v_e (or at the cell before v_s's first base when v_e =
    v_s and the walk starts at offset 0, as the extension form's end rule
    has it), scored by edit distance to q.  Returns (d, set of
    end offsets in v_e reaching d), (-1, set()) when v_e cannot be reached.
    Walks longer than |q| + max(|q|, S) bases, S the shortest spelled length
    that reaches the first base of v_e, cannot be optimal, which bounds the
    enumeration on cyclic graphs."""
    import heapq
    if j1 is None:
        j1 = j0
    q = (q.decode() if isinstance(q, (bytes, bytearray)) else q).upper()
    n = len(q)
    succ = {}
    for a, b in edges:
        succ.setdefault(a, []).append(b)
    # shortest spelled length before the first base of each vertex (start: j0)
    dist = {}
    pq = [(0, v_s)]
    seen = set()
    while pq:
        d, v = heapq.heappop(pq)
        if v in seen:
            continue
        seen.add(v)
        dist[v] = d
        stay = len(labels[v]) - (j0 if (v == v_s and d == 0) else 0)
        for u in succ.get(v, []):
            if u not in seen:
                heapq.heappush(pq, (d + stay, u))
    if v_e not in dist:
        return -1, set()
    limit = n + max(n, dist[v_e] + 1)
    best = [1 << 60]
    ends = set()
    qa = list(q)

    def note(d, j):
        if d < best[0]:
            best[0] = d
            ends.clear()
        if d == best[0]:
            ends.add(j)

    def step(col, c):
        new = [col[0] + 1]
        for i in range(1, n + 1):
            new.append(min(col[i - 1] + (qa[i - 1] != c), col[i] + 1, new[i - 1] + 1))
        return new

    def dfs(v, col, depth, first=0):
        lab = labels[v].upper()
        for j in range(first, len(lab)):
            col = step(col, lab[j])
            depth += 1
            if v == v_e:
                note(col[n], j + 1)
            # as in the extension form, the cell before v_s's first base holds
            # this value too when the walk can step from here into v_s, and it
            # is an end cell when the walk started there
            if j + 1 == len(lab) and v_e == v_s and j0 == 0 and v_s in succ.get(v, []):
                note(col[n], 0)
            if depth > limit or min(col) > best[0]:
                return
        for u in succ.get(v, []):
            dfs(u, col, depth)

    for j in range(j0, j1 + 1):
        if v_s == v_e and (j >= 1 or j0 == 0):
            note(n, j)          # the start cell itself: nothing of the walk spelled
        dfs(v_s, list(range(n + 1)), 0, j)
    return best[0], ends


def mutate(rng, s: bytes, err: float) -> bytes:
    """Substitutions, insertions and deletions, each at rate err/3 per base."""
    out = bytearray()
    for c in s:
        r = rng.random()
        if r < err / 3:
            out.append(b"ACGT"[(b"ACGT".index(c) + 1 + int(rng.integers(0, 3))) % 4])
        elif r < 2 * err / 3:
            out.append(c)
            out.append(b"ACGT"[int(rng.integers(0, 4))])
        elif r < err:
            pass
        else:
            out.append(c)
    return bytes(out)


def medium_case(rng):
    """A 20-200 vertex graph (labels mostly 1-8 bases, some up to 400; a
    backbone chain, skip edges forming bubbles, back edges and self-loops
    forming cycles) and a query spelled along a random walk of 50-3,000 bases
    with 0-12% errors.  Returns (labels, edges, q, v_s, last vertex of the
    walk)."""
    n = int(rng.integers(20, 200))
    lens = []
    for _ in range(n):
        u = rng.random()
        lens.append(int(rng.integers(1, 9)) if u < 0.7 else
                    (int(rng.integers(9, 61)) if u < 0.95 else int(rng.integers(61, 401))))
    labels = ["".join("ACGT"[x] for x in rng.integers(0, 4, size=L)) for L in lens]
    edges = set((a, a + 1) for a in range(n - 1))
    for a in range(n):
        if rng.random() < 0.3 and a + 2 < n:
            edges.add((a, int(rng.integers(a + 2, min(n, a + 6)))))
        if rng.random() < 0.08 and a > 0:
            edges.add((a, int(rng.integers(max(0, a - 30), a))))
        if rng.random() < 0.03:
            edges.add((a, a))
    edges = sorted(edges)
    vs = int(rng.integers(0, n // 2))
    t, walk = spell_random_walk(rng, labels, edges, vs, int(rng.integers(50, 3000)))
    return labels, edges, mutate(rng, t, float(rng.uniform(0.0, 0.12))), vs, walk[-1]


# ---------------------------------------------------------------------------
# An independent pairwise wavefront with the pruning rule of Algorithm 4, for
# graphs whose every walk from the start has the same length up to each base
# (chains; SNP bubbles of two one-base alleles).  There the aligned walk
# length W~ of a front cell is its position in the walk, so Algorithm 4's
# quantity a = i + W~ is the textbook a = i + j of a pairwise alignment and
# the graph transcription must give the same distance and end position.
# ---------------------------------------------------------------------------
def pairwise_wf_pruned(q: bytes, cols, a_diff: int = 0):
    """Extension-form alignment of q against a prefix of the column string
    `cols` (cols[j] = the set of bases allowed at position j), by furthest-
    reaching diagonals d = j - i (i query bases, j columns consumed).  Per
    score: extend every diagonal by its exact-match run; stop when some
    diagonal has consumed q (end = the smallest such j); if the largest
    a = i + j exceeds a_diff, keep only diagonals with a_max - a < a_diff
    (a dropped diagonal keeps its furthest point as its record); then expand
    by insertion (i+1), deletion (j+1) and mismatch (both), per diagonal the
    furthest candidate, admitted only past the diagonal's record.
    Returns (distance, end j)."""
    q = q.upper()
    n, m = len(q), len(cols)
    rec = {}
    wf = {0: 0}
    s = 0
    while True:
        for dg in list(wf):
            i = wf[dg]
            while i < n and i + dg < m and q[i] in cols[i + dg]:
                i += 1
            wf[dg] = i
            rec[dg] = i
        ends = [i + dg for dg, i in wf.items() if i == n]
        if ends:
            return s, min(ends)
        if a_diff > 0:
            amax = max(2 * i + dg for dg, i in wf.items())
            if amax > a_diff:
                wf = {dg: i for dg, i in wf.items() if amax - (2 * i + dg) < a_diff}
        nxt = {}
        for dg, i in wf.items():
            j = i + dg
            cand = []
            if i < n:
                cand.append((dg - 1, i + 1))          # query base alone
            if j < m:
                cand.append((dg + 1, i))              # column alone
            if i < n and j < m:
                cand.append((dg, i + 1))              # substitution
            for nd, ni in cand:
                if nd in rec and rec[nd] >= ni:
                    continue
                if ni > nxt.get(nd, -1):
                    nxt[nd] = ni
        wf = nxt
        s += 1


def chain_case(rng, length: int, max_piece: int):
    """A random string cut at random points into a chain of vertices.
    Returns (labels, edges, column sets, backbone position of each vertex)."""
    t = "".join("ACGT"[x] for x in rng.integers(0, 4, size=length))
    labels, pos, p = [], [], 0
    while p < length:
        c = int(rng.integers(1, max_piece + 1))
        labels.append(t[p:p + c])
        pos.append(p)
        p += c
    edges = [(a, a + 1) for a in range(len(labels) - 1)]
    return labels, edges, [frozenset(ch.encode()) for ch in t], pos


def snp_bubble_case(rng, length: int, snp_rate: float, max_piece: int):
    """A backbone with SNP bubbles (two one-base alleles with different
    bases) cut into vertices in topological order.  Returns (labels, edges,
    column sets, backbone position of each vertex, backbone string)."""
    labels, pos, edges, cols = [], [], [], []
    tails = []
    p = 0
    while p < length:
        if p > 0 and rng.random() < snp_rate:
            a = "ACGT"[int(rng.integers(0, 4))]
            b = "ACGT"[("ACGT".index(a) + int(rng.integers(1, 4))) % 4]
            ids = []
            for x in (a, b):
                labels.append(x)
                pos.append(p)
                ids.append(len(labels) - 1)
                edges += [(t, ids[-1]) for t in tails]
            tails = ids
            cols.append(frozenset((a + b).encode()))
            p += 1
        else:
            c = int(min(rng.integers(1, max_piece + 1), length - p))
            s = "".join("ACGT"[x] for x in rng.integers(0, 4, size=c))
            labels.append(s)
            pos.append(p)
            v = len(labels) - 1
            edges += [(t, v) for t in tails]
            tails = [v]
            cols += [frozenset(ch.encode()) for ch in s]
            p += c
    return labels, edges, cols, pos


def spell_cols(rng, cols) -> bytes:
    """One string through the column sets (a random allowed base each)."""
    out = bytearray()
    for c in cols:
        c = sorted(c)
        out.append(c[int(rng.integers(0, len(c)))])
    return bytes(out)


# ---------------------------------------------------------------------------
# Walk lengths W~ on graphs whose walks differ in length (indels, loops).
#
# (1) A soundness reference from Eq. 1 with the walk length as an extra
#     index: C[i][w][p] = the least cost of aligning q[1..i] to a walk string
#     of exactly w bases that starts at the start cell and ends at base
#     position p.  A front cell reached at score s along a chain of
#     expansions (cost 1) and extensions / crossings (cost 0) has a walk of
#     length W~ with an alignment of cost s, so C[i][W~][p] <= s; in the
#     exact form the front cell's Eq. 1 value is s, so equality holds.
# (2) The tie rules of the reading of W~ (the larger W~ between candidates
#     of one diagonal with the same offset; crossings grouped in rounds, the
#     larger W~ within a round, an earlier round first) re-implemented with
#     per-score dictionaries and explicit crossing layers.
# ---------------------------------------------------------------------------
def walk_length_costs(labels, edges, q: bytes, v_s: int, w_max: int, j0: int = 0):
    """Returns (C, pos) with C of shape (|q|+1, w_max+1, P+1): P base
    positions (v, j), j = 1..|v|, indexed by pos[(v, j)], and index P the
    start when j0 = 0 (with j0 >= 1 the start is the position (v_s, j0))."""
    q = q.upper()
    labs = [l.upper() for l in labels]
    pos = {}
    for v, s in enumerate(labs):
        for j in range(1, len(s) + 1):
            pos[(v, j)] = len(pos)
    P = len(pos)
    start = P if j0 == 0 else pos[(v_s, j0)]
    INF = 1 << 30
    preds = [[] for _ in range(P)]
    base = np.zeros(P, dtype=np.uint8)
    for (v, j), p in pos.items():
        base[p] = ord(labs[v][j - 1])
        if j >= 2:
            preds[p].append(pos[(v, j - 1)])
        else:
            preds[p] += [pos[(u, len(labs[u]))] for u, b in edges if b == v]
            if v == v_s and j0 == 0:
                preds[p].append(P)
    width = max(1, max(len(x) for x in preds))
    pm = np.full((P, width), P + 1, dtype=np.int64)     # P + 1: an always-infinite pad slot
    for p, x in enumerate(preds):
        pm[p, :len(x)] = sorted(set(x))
    n = len(q)
    C = np.full((n + 1, w_max + 1, P + 2), INF, dtype=np.int64)
    C[0, 0, start] = 0
    qa = np.frombuffer(q, dtype=np.uint8)
    for i in range(n + 1):
        for w in range(w_max + 1):
            row = C[i, w]
            if i > 0:
                np.minimum(row, C[i - 1, w] + 1, out=row)                       # query base alone
            if w > 0:
                prev = C[i, w - 1][pm].min(axis=1)
                np.minimum(row[:P], prev + 1, out=row[:P])                       # walk base alone
                if i > 0:
                    diag = C[i - 1, w - 1][pm].min(axis=1) + (base != qa[i - 1])
                    np.minimum(row[:P], diag, out=row[:P])                       # match / substitution
            row[P + 1] = INF
    return C[:, :, :P + 1], pos


def front_cell_cost(C, pos, labels, edges, v_s: int, j0: int, i: int, v: int, off: int, W: int) -> int:
    """Least cost over walks of exactly W bases ending at the front cell
    (v, off): the base position (v, off) when off >= 1; with off = 0 the last
    base of a predecessor of v, or the empty walk at the start."""
    if W >= C.shape[1]:
        return 1 << 30
    if off >= 1:
        return int(C[i, W, pos[(v, off)]])
    cands = [pos[(u, len(labels[u]))] for u, b in edges if b == v]
    if v == v_s and j0 == 0:
        cands.append(C.shape[2] - 1)
    return min((int(C[i, W, p]) for p in cands), default=1 << 30)


def gwf_walk_lengths(labels, edges, q: bytes, v_s: int, a_diff: int = 0, j0: int = 0, variant: str = ""):
    """Algorithms 1-4 (extension form) with the walk length W~ of each
    diagonal, written with one dictionary per score and explicit crossing
    layers.  Returns (distance, end (v, j), entries) with entries the
    sorted (score, v, k, offset, W~) of every extended wavefront.

    `variant` swaps one rule for a plausible alternative, to show that the
    inputs exercise each rule: "min_w" (the smaller W~ on offset ties and
    within a round), "first_w" (the first crossing of a round into a
    diagonal sets its W~), "lifo" (crossings followed depth first, no
    rounds: the first path to reach a diagonal sets its W~), "ins_w" (an
    insertion advances W~)."""
    q = q.upper()
    labs = [l.upper() for l in labels]
    succ = {}
    for a, b in edges:
        succ.setdefault(a, []).append(b)
    n = len(q)
    better = (lambda x, y: x < y) if variant == "min_w" else (lambda x, y: x > y)
    rec = {(v_s, -j0): j0}                # diagonal -> furthest offset (kept for the query's life)
    wave = {(v_s, -j0): (j0, 0)}          # this score's diagonals before extension: (offset, W~)
    entries = []
    s = 0
    while True:
        ext = {}

        def extend(v, k, o, W):
            lab = labs[v]
            while k + o < n and o < len(lab) and q[k + o] == ord(lab[o]):
                o += 1
                W += 1
            ext[(v, k)] = (o, W)
            rec[(v, k)] = o
            return o, W

        if variant == "lifo":
            stack = list(wave.items())[::-1]
            while stack:
                (v, k), (o, W) = stack.pop()
                o, W = extend(v, k, o, W)
                if o == len(labs[v]):
                    for u in reversed(succ.get(v, [])):
                        t = (u, k + len(labs[v]))
                        if t not in rec:
                            rec[t] = 0
                            stack.append((t, (0, W)))
        layer = {} if variant == "lifo" else wave
        while layer:
            for (v, k), (o, W) in layer.items():
                extend(v, k, o, W)
            nxt = {}
            for (v, k) in layer:
                o, W = ext[(v, k)]
                if o != len(labs[v]):
                    continue
                for u in succ.get(v, []):
                    t = (u, k + len(labs[v]))
                    if t in rec:
                        continue
                    if t not in nxt or (variant != "first_w" and better(W, nxt[t])):
                        nxt[t] = W
            for t in nxt:
                rec[t] = 0
            layer = {t: (0, W) for t, W in nxt.items()}
        entries += [(s, v, k, o, W) for (v, k), (o, W) in ext.items()]
        ends = [(v, o) for (v, k), (o, W) in ext.items()
                if k + o == n and (o > 0 or (v == v_s and j0 == 0))]
        if ends:
            return s, min(ends), sorted(entries)
        keep = ext
        if a_diff > 0:
            amax = max([0] + [k + o + W for (v, k), (o, W) in ext.items()])
            if amax > a_diff:
                keep = {d: x for d, x in ext.items() if amax - (d[1] + x[0] + x[1]) < a_diff}
        cand = {}
        for (v, k), (o, W) in keep.items():
            L = len(labs[v])
            c = []
            if k + o < n:
                c.append(((v, k + 1), o, W + (1 if variant == "ins_w" else 0)))
            if o < L:
                c.append(((v, k - 1), o + 1, W + 1))
            if k + o < n and o < L:
                c.append(((v, k), o + 1, W + 1))
            for d, no, nw in c:
                if rec.get(d, -1) >= no:
                    continue
                if d not in cand or no > cand[d][0] or (no == cand[d][0] and better(nw, cand[d][1])):
                    cand[d] = (no, nw)
        for d, (no, nw) in cand.items():
            rec[d] = no
        wave = cand
        s += 1
