/*
 * oracle.c -- plain CPU oracle for graph wavefront alignment (Gwfa).
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only code that may load this
 * library.  The product path (the HIP library and its Python binding) never
 * calls it, links it or shares any code with it.
 *
 * Everything here is deliberately slow and written to be checked by eye
 * against the paper (Zhang, Wu, Aluru, Li: "Fast sequence to graph
 * alignment using the graph wavefront algorithm"):
 *
 *   orc_dp_dense    Eq. 1 (Section 2.2) cell by cell, one query row at a
 *                   time, with the in-row terms (deletion inside a vertex,
 *                   zero-cost carry over an edge) iterated to a fixpoint,
 *                   which is unique because labels are non-empty (Section 2.2
 *                   cites the uniqueness result for cyclic recurrences).
 *   orc_dp_capped   The same recurrence with every value saturated at D+1;
 *                   only cells <= D are stored.  Exact whenever d* <= D.
 *   orc_ed_global   Textbook pairwise edit distance (used to re-score walks).
 *   orc_ed_banded   The same restricted to |i-j| <= D (exact when ED <= D).
 *   orc_dp_dense_global  The same rows; the answer is the cell
 *                   H_{|q|, v_e, |v_e|} (the global form with an end vertex).
 *   orc_dp_dense_clip  The same with a free end gap in the query (up to e
 *                   trailing bases left unaligned at no cost): the best
 *                   over rows |q| - e .. |q|.
 *   wfree           (orc_dp_dense_at, orc_dp_dense_clip, orc_gwf) the global
 *                   form with a free end gap in the walk (one of the
 *                   variants Section 2.2 points to): the walk may end
 *                   anywhere inside v_e, so the answer is the best cell
 *                   (|q|, v_e, j) over j >= 1 (plus j = 0 when v_e = v_s and
 *                   the walk starts at offset 0), the smallest j on ties.
 *   orc_dp_dense_at Either form with the walk starting after the first j0
 *                   bases of v_s: the initial condition moves to
 *                   H_{0, v_s, j0} = 0 (a read seeded inside a vertex); with
 *                   a window j0..j1, H_{0, v_s, j} = 0 for all of it (the
 *                   walk's leading gap in v_s is free).
 *   orc_gwf         Algorithms 1-4 (Sections 2.4-2.5): the wavefront
 *                   driver, extension, expansion and the pruning heuristic,
 *                   in extension mode or, with an end vertex, the global
 *                   form.  This is the oracle for the pruning heuristic and
 *                   for wavefront work counts.  Pinned with pruning on
 *                   graphs whose walks from the start all have the same
 *                   length up to each base (there W~ is the walk position
 *                   and an independent pairwise wavefront with the same
 *                   keep rule must agree).  Where walks differ in length,
 *                   every W~ is pinned as the length of a real walk that
 *                   aligns the consumed query prefix at no more than the
 *                   entry's score (Eq. 1 with the walk length as an extra
 *                   index), and the tie rules between such walks (a choice
 *                   the paper leaves open) against an independent
 *                   implementation of the same rules.
 *   orc_rev_dp      Reverse form of Eq. 1 (cost to finish from a cell), used
 *                   to label wavefront entries for the learned pruning.
 *
 * Problem (Def. 2.2 in extension mode, no end vertex): the query q must be
 * consumed entirely; the walk starts before the first base of v_s; the end
 * is free anywhere in the graph.  d* = min over the last query row.
 * End position: lexicographic minimum (v, j) over last-row cells equal to
 * d* with j >= 1, plus (v_s, 0) when that cell equals d*.  With a start
 * offset j0 > 0 the start cell is (v_s, j0), already a j >= 1 cell, and
 * (v_s, 0) is an ordinary j = 0 cell (not an end).
 *
 * Sequences are ASCII; bases compare case-insensitively.  Input validation
 * (alphabet, ranges) is the caller's job: the oracle assumes valid input.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define INF_H (INT32_MAX / 4)

static inline uint8_t up(uint8_t c) { return (c >= 'a' && c <= 'z') ? (uint8_t)(c - 32) : c; }

/* ------------------------------------------------------------------ */
/* graph helpers                                                        */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t n;
    const uint8_t *seq;
    const int64_t *off;   /* n+1 */
    int64_t ncell;        /* sum(|v|+1) */
    int64_t *base;        /* first cell of v: off[v] + v */
    int32_t *in_off, *in_src;    /* in-edge CSR */
    int32_t *out_off, *out_dst;  /* out-edge CSR */
    int32_t *cell_v;      /* cell -> vertex */
} ograph;

static int64_t vlen(const ograph *g, int32_t v) { return g->off[v + 1] - g->off[v]; }

static int graph_init(ograph *g, int32_t n, const uint8_t *seq, const int64_t *off,
                      int64_t ne, const int32_t *src, const int32_t *dst, int need_cell_v)
{
    memset(g, 0, sizeof(*g));
    g->n = n; g->seq = seq; g->off = off;
    g->base = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    g->in_off = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    g->out_off = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    g->in_src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    g->out_dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    if (!g->base || !g->in_off || !g->out_off || !g->in_src || !g->out_dst) return -1;
    for (int32_t v = 0; v <= n; v++) g->base[v] = off[v] + v;
    g->ncell = g->base[n];
    for (int64_t e = 0; e < ne; e++) { g->in_off[dst[e] + 1]++; g->out_off[src[e] + 1]++; }
    for (int32_t v = 0; v < n; v++) { g->in_off[v + 1] += g->in_off[v]; g->out_off[v + 1] += g->out_off[v]; }
    int32_t *fi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *fo = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!fi || !fo) { free(fi); free(fo); return -1; }
    memcpy(fi, g->in_off, sizeof(int32_t) * (size_t)(n + 1));
    memcpy(fo, g->out_off, sizeof(int32_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < ne; e++) {   /* edges kept in input order */
        g->in_src[fi[dst[e]]++] = src[e];
        g->out_dst[fo[src[e]]++] = dst[e];
    }
    free(fi); free(fo);
    if (need_cell_v) {
        g->cell_v = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->ncell > 0 ? g->ncell : 1));
        if (!g->cell_v) return -1;
        for (int32_t v = 0; v < n; v++)
            for (int64_t c = g->base[v]; c < g->base[v + 1]; c++) g->cell_v[c] = v;
    }
    return 0;
}

static void graph_free(ograph *g)
{
    free(g->base); free(g->in_off); free(g->in_src); free(g->out_off); free(g->out_dst); free(g->cell_v);
}

/* ------------------------------------------------------------------ */
/* Eq. 1, dense                                                         */
/* ------------------------------------------------------------------ */

/* In-row terms of Eq. 1 (fourth case: carry H_{i,u,|u|} onto (v,0) for
 * every in-edge (u,v); second case: H_{i,v,j-1}+1), swept over the vertices
 * in id order until nothing changes.  Returns the number of sweeps, or -1
 * when it fails to converge within |V|+2 sweeps (impossible for non-empty
 * labels: a shortest in-row chain visits each vertex at most once). */
static int row_fixpoint(const ograph *g, int32_t *h)
{
    int sweeps = 0, changed;
    do {
        changed = 0;
        sweeps++;
        if (sweeps > g->n + 2) return -1;
        for (int32_t v = 0; v < g->n; v++) {
            int64_t c0 = g->base[v];
            for (int32_t e = g->in_off[v]; e < g->in_off[v + 1]; e++) {
                int32_t u = g->in_src[e];
                int32_t x = h[g->base[u] + vlen(g, u)];
                if (x < h[c0]) { h[c0] = x; changed = 1; }
            }
            int64_t L = vlen(g, v);
            for (int64_t j = 1; j <= L; j++)
                if (h[c0 + j - 1] + 1 < h[c0 + j]) { h[c0 + j] = h[c0 + j - 1] + 1; changed = 1; }
        }
    } while (changed);
    return sweeps;
}

/* Reads the answer off the last row: d* = row minimum; end = lexicographic
 * minimum (v,j) among cells equal to d* with j >= 1, or (v_s,0). */
/* End of the extension form: lexicographically smallest (v, j) holding the
 * row minimum, over cells with j >= 1 plus the start cell (v_s, 0) when the
 * walk starts at offset 0 (a cell (v, 0) otherwise ties with the end cell of
 * a predecessor). */
static void row_answer(const ograph *g, const int32_t *h, int32_t v_s, int32_t j0, int32_t *out)
{
    int32_t best = INF_H;
    for (int64_t c = 0; c < g->ncell; c++) if (h[c] < best) best = h[c];
    out[0] = best; out[1] = -1; out[2] = -1;
    for (int32_t v = 0; v < g->n; v++) {
        int64_t L = vlen(g, v);
        for (int64_t j = 0; j <= L; j++) {
            if (j == 0 && !(v == v_s && j0 == 0)) continue;
            if (h[g->base[v] + j] == best) { out[1] = v; out[2] = (int32_t)j; return; }
        }
    }
}

/* Global form with a free end gap in the walk: the best cell of v_e's row
 * segment, over j >= 1 plus (v_e, 0) when v_e is the start vertex and the
 * walk starts at offset 0 (as in row_answer, a cell (v, 0) is otherwise the
 * copy of a predecessor's last cell, which lies outside v_e); the smallest
 * j on ties.  out[0] = INF_H when no cell of v_e is reached. */
static void row_answer_in(const ograph *g, const int32_t *h, int32_t v_e, int32_t v_s, int32_t j0, int32_t *out)
{
    out[0] = INF_H; out[1] = v_e; out[2] = (int32_t)vlen(g, v_e);
    for (int64_t j = 0; j <= vlen(g, v_e); j++) {
        if (j == 0 && !(v_e == v_s && j0 == 0)) continue;
        if (h[g->base[v_e] + j] < out[0]) { out[0] = h[g->base[v_e] + j]; out[2] = (int32_t)j; }
    }
}

/* out[0]=d*, out[1]=end vertex, out[2]=end offset j, out[3]=max sweeps in a row.
 * Returns 0, or -1 on allocation failure / non-convergence. */
/* Called with every finished row i >= row_lo (after its fixpoint). */
typedef void (*row_fn)(void *cb, const ograph *g, int32_t i, const int32_t *h);

/* Rows 0..|q| of Eq. 1; returns the last row (caller frees) or NULL. */
static int32_t *dense_rows(const ograph *g, const uint8_t *q, int32_t qlen, int32_t v_s, int32_t j0,
                           int32_t j1, int32_t row_lo, row_fn fn, void *cb, int *maxsw_out)
{
    int32_t n = g->n;
    const uint8_t *seq = g->seq;
    const int64_t *off = g->off;
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->ncell);
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->ncell);
    if (!prev || !cur) { free(prev); free(cur); return NULL; }
    int maxsw = 0, rc = 0;
    /* row 0: initial condition H_{0,v_s,j} = 0 for j0 <= j <= j1 (j0 = j1 =
     * 0: the paper's H_{0,v_s,0}; j0 > 0 starts after the first j0 bases of
     * v_s; j1 > j0 leaves the walk's start free in that window), everything
     * else infinite */
    for (int64_t c = 0; c < g->ncell; c++) prev[c] = INF_H;
    for (int32_t j = j0; j <= j1; j++) prev[g->base[v_s] + j] = 0;
    int sw = row_fixpoint(g, prev);
    if (sw < 0) rc = -1; else if (sw > maxsw) maxsw = sw;
    if (rc == 0 && fn && row_lo <= 0) fn(cb, g, 0, prev);
    for (int32_t i = 1; i <= qlen && rc == 0; i++) {
        uint8_t qi = up(q[i - 1]);
        for (int32_t v = 0; v < n; v++) {
            int64_t c0 = g->base[v], L = vlen(g, v);
            const uint8_t *lab = seq + off[v];
            for (int64_t j = 0; j <= L; j++) {
                int32_t h = prev[c0 + j] + 1;                      /* first case: consume q[i] only */
                if (j >= 1) {                                      /* third case: (mis)match q[i] with v[j] */
                    int32_t dlt = (qi == up(lab[j - 1])) ? 0 : 1;
                    int32_t x = prev[c0 + j - 1] + dlt;
                    if (x < h) h = x;
                }
                cur[c0 + j] = h < INF_H ? h : INF_H;
            }
        }
        sw = row_fixpoint(g, cur);
        if (sw < 0) rc = -1; else if (sw > maxsw) maxsw = sw;
        if (rc == 0 && fn && i >= row_lo) fn(cb, g, i, cur);
        int32_t *t = prev; prev = cur; cur = t;
    }
    free(cur);
    if (rc) { free(prev); return NULL; }
    *maxsw_out = maxsw;
    return prev;
}

static int32_t *dense_last_row(const ograph *g, const uint8_t *q, int32_t qlen, int32_t v_s, int32_t j0,
                               int32_t j1, int *maxsw_out)
{
    return dense_rows(g, q, qlen, v_s, j0, j1, qlen + 1, NULL, NULL, maxsw_out);
}

/* Free end gap in the query: the best over rows i >= |q| - e (the last
 * |q| - i query bases left unaligned at no cost).  The distance is the
 * smallest row value; among rows that reach it the largest i wins (the
 * fewest unaligned bases), then the row's own end rule. */
typedef struct {
    int32_t v_s, j0, v_e, wfree;
    int32_t d, ev, ej, i;     /* best so far; d = INF_H: none */
} clip_best;

static void clip_row(void *cbv, const ograph *g, int32_t i, const int32_t *h)
{
    clip_best *cb = (clip_best *)cbv;
    int32_t o[3];
    if (cb->v_e >= 0 && cb->wfree) {
        row_answer_in(g, h, cb->v_e, cb->v_s, cb->j0, o);
    } else if (cb->v_e >= 0) {
        int32_t Le = (int32_t)vlen(g, cb->v_e);
        o[0] = h[g->base[cb->v_e] + Le]; o[1] = cb->v_e; o[2] = Le;
    } else {
        row_answer(g, h, cb->v_s, cb->j0, o);
    }
    if (o[0] < INF_H && o[0] <= cb->d) {   /* rows come in increasing i: ties go to the later row */
        cb->d = o[0]; cb->ev = o[1]; cb->ej = o[2]; cb->i = i;
    }
}

int orc_dp_dense(int32_t n, const uint8_t *seq, const int64_t *off, int64_t ne,
                 const int32_t *src, const int32_t *dst,
                 const uint8_t *q, int32_t qlen, int32_t v_s, int32_t *out)
{
    ograph g;
    if (graph_init(&g, n, seq, off, ne, src, dst, 0)) { graph_free(&g); return -1; }
    int maxsw = 0;
    int32_t *last = dense_last_row(&g, q, qlen, v_s, 0, 0, &maxsw);
    if (!last) { graph_free(&g); return -1; }
    row_answer(&g, last, v_s, 0, out);
    out[3] = maxsw;
    free(last); graph_free(&g);
    return 0;
}

/* The same with the walk starting after the first j (j0 <= j <= j1 <=
 * |v_s|, free within the window; j1 < 0 means j1 = j0) bases of v_s and,
 * when v_e >= 0, the global form: out[0] is then H_{|q|, v_e, |v_e|} (-1
 * when unreachable), out[1] = v_e, out[2] = |v_e|; with wfree, the best
 * cell of v_e (row_answer_in) and its offset. */
int orc_dp_dense_at(int32_t n, const uint8_t *seq, const int64_t *off, int64_t ne,
                    const int32_t *src, const int32_t *dst,
                    const uint8_t *q, int32_t qlen, int32_t v_s, int32_t j0, int32_t j1, int32_t v_e, int32_t wfree,
                    int32_t *out)
{
    ograph g;
    if (graph_init(&g, n, seq, off, ne, src, dst, 0)) { graph_free(&g); return -1; }
    if (j1 < 0) j1 = j0;
    if (v_s < 0 || v_s >= n || v_e >= n || j0 < 0 || j1 < j0 || j1 > vlen(&g, v_s)) { graph_free(&g); return -1; }
    int maxsw = 0;
    int32_t *last = dense_last_row(&g, q, qlen, v_s, j0, j1, &maxsw);
    if (!last) { graph_free(&g); return -1; }
    if (v_e < 0) {
        row_answer(&g, last, v_s, j0, out);
    } else if (wfree) {
        row_answer_in(&g, last, v_e, v_s, j0, out);
        if (out[0] >= INF_H) { out[0] = -1; out[2] = (int32_t)vlen(&g, v_e); }
    } else {
        int32_t h = last[g.base[v_e] + vlen(&g, v_e)];
        out[0] = h >= INF_H ? -1 : h; out[1] = v_e; out[2] = (int32_t)vlen(&g, v_e);
    }
    out[3] = maxsw;
    free(last); graph_free(&g);
    return 0;
}

/* orc_dp_dense_at with a free end gap of up to e query bases (0 <= e <=
 * |q|): out[0] = distance (-1 when the global form's end vertex is
 * unreachable), out[1..2] = end (v, j), out[3] = |q| - i of the chosen row
 * (query bases left unaligned). */
int orc_dp_dense_clip(int32_t n, const uint8_t *seq, const int64_t *off, int64_t ne,
                      const int32_t *src, const int32_t *dst,
                      const uint8_t *q, int32_t qlen, int32_t v_s, int32_t j0, int32_t j1, int32_t v_e,
                      int32_t wfree, int32_t e, int32_t *out)
{
    ograph g;
    if (graph_init(&g, n, seq, off, ne, src, dst, 0)) { graph_free(&g); return -1; }
    if (j1 < 0) j1 = j0;
    if (v_s < 0 || v_s >= n || v_e >= n || j0 < 0 || j1 < j0 || j1 > vlen(&g, v_s) || e < 0 || e > qlen) {
        graph_free(&g);
        return -1;
    }
    clip_best cb = {v_s, j0, v_e, wfree, INF_H, -1, -1, -1};
    int maxsw = 0;
    int32_t *last = dense_rows(&g, q, qlen, v_s, j0, j1, qlen - e, clip_row, &cb, &maxsw);
    if (!last) { graph_free(&g); return -1; }
    if (cb.d >= INF_H) { out[0] = -1; out[1] = v_e; out[2] = v_e >= 0 ? (int32_t)vlen(&g, v_e) : -1; out[3] = 0; }
    else { out[0] = cb.d; out[1] = cb.ev; out[2] = cb.ej; out[3] = qlen - cb.i; }
    free(last); graph_free(&g);
    return 0;
}

/* Global form of Definition 2.2: the walk runs from before the first base of
 * v_s to the last base of v_e; the distance is H_{|q|, v_e, |v_e|} of Eq. 1
 * (out[0]; -1 when no walk from v_s reaches v_e). */
int orc_dp_dense_global(int32_t n, const uint8_t *seq, const int64_t *off, int64_t ne,
                        const int32_t *src, const int32_t *dst,
                        const uint8_t *q, int32_t qlen, int32_t v_s, int32_t v_e, int32_t *out)
{
    ograph g;
    if (graph_init(&g, n, seq, off, ne, src, dst, 0)) { graph_free(&g); return -1; }
    int maxsw = 0;
    int32_t *last = dense_last_row(&g, q, qlen, v_s, 0, 0, &maxsw);
    if (!last) { graph_free(&g); return -1; }
    int32_t h = last[g.base[v_e] + vlen(&g, v_e)];
    out[0] = h >= INF_H ? -1 : h;
    out[1] = maxsw;
    free(last); graph_free(&g);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Eq. 1, value-capped                                                  */
/* ------------------------------------------------------------------ */
typedef struct { int64_t *a; int64_t n, cap; } vec64;
static int v_push(vec64 *v, int64_t x)
{
    if (v->n == v->cap) {
        int64_t nc = v->cap ? v->cap * 2 : 64;
        int64_t *na = (int64_t *)realloc(v->a, sizeof(int64_t) * (size_t)nc);
        if (!na) return -1;
        v->a = na; v->cap = nc;
    }
    v->a[v->n++] = x;
    return 0;
}

typedef struct {
    int32_t D;
    int32_t *val;       /* per cell; INF_H when > D */
    vec64 live;         /* cells with val <= D */
    vec64 *bucket;      /* D+1 buckets */
    int err;
} caprow;

static inline void cap_relax(caprow *r, int64_t c, int32_t x)
{
    if (x > r->D || x >= r->val[c]) return;
    if (r->val[c] >= INF_H) r->err |= v_push(&r->live, c);
    r->val[c] = x;
    r->err |= v_push(&r->bucket[x], c);
}

/* The in-row terms of Eq. 1 restricted to values <= D.  The row is the least
 * solution of h = min(h0, deletion +1 inside a vertex, carry +0 over an edge);
 * all move costs are 0 or 1, so visiting cells in non-decreasing value
 * (a bucket queue) settles every cell at that least solution. */
static void cap_closure(const ograph *g, caprow *r)
{
    for (int32_t b = 0; b <= r->D; b++) {
        for (int64_t p = 0; p < r->bucket[b].n; p++) {
            int64_t c = r->bucket[b].a[p];
            if (r->val[c] != b) continue;              /* superseded */
            int32_t v = g->cell_v[c];
            int64_t j = c - g->base[v];
            if (j < vlen(g, v)) cap_relax(r, c + 1, b + 1);
            else
                for (int32_t e = g->out_off[v]; e < g->out_off[v + 1]; e++)
                    cap_relax(r, g->base[g->out_dst[e]], b);
        }
        r->bucket[b].n = 0;
    }
}

/* out[0] = d* (or -1 when d* > D), out[1], out[2] = end (v, j). */
int orc_dp_capped(int32_t n, const uint8_t *seq, const int64_t *off, int64_t ne,
                  const int32_t *src, const int32_t *dst,
                  const uint8_t *q, int32_t qlen, int32_t v_s, int32_t D, int32_t *out)
{
    ograph g;
    if (D < 0) return -1;
    if (graph_init(&g, n, seq, off, ne, src, dst, 1)) { graph_free(&g); return -1; }
    caprow A, B;
    memset(&A, 0, sizeof(A)); memset(&B, 0, sizeof(B));
    A.D = B.D = D;
    A.val = (int32_t *)malloc(sizeof(int32_t) * (size_t)g.ncell);
    B.val = (int32_t *)malloc(sizeof(int32_t) * (size_t)g.ncell);
    vec64 *bk = (vec64 *)calloc((size_t)D + 1, sizeof(vec64));
    int rc = 0;
    if (!A.val || !B.val || !bk) { rc = -1; goto done; }
    A.bucket = B.bucket = bk;
    for (int64_t c = 0; c < g.ncell; c++) A.val[c] = B.val[c] = INF_H;
    caprow *prev = &A, *cur = &B;
    cap_relax(prev, g.base[v_s], 0);                   /* H_{0,v_s,0} = 0 */
    cap_closure(&g, prev);
    for (int32_t i = 1; i <= qlen; i++) {
        uint8_t qi = up(q[i - 1]);
        for (int64_t p = 0; p < prev->live.n; p++) {
            int64_t c = prev->live.a[p];
            int32_t h = prev->val[c];
            int32_t v = g.cell_v[c];
            int64_t j = c - g.base[v];
            cap_relax(cur, c, h + 1);                  /* first case */
            if (j < vlen(&g, v)) {                     /* third case into (v, j+1) */
                int32_t dlt = (qi == up(seq[off[v] + j])) ? 0 : 1;
                cap_relax(cur, c + 1, h + dlt);
            }
        }
        cap_closure(&g, cur);
        for (int64_t p = 0; p < prev->live.n; p++) prev->val[prev->live.a[p]] = INF_H;
        prev->live.n = 0;
        caprow *t = prev; prev = cur; cur = t;
        if (prev->err || cur->err) { rc = -1; goto done; }
        if (prev->live.n == 0) break;                  /* every cell saturated: d* > D */
    }
    {
        int32_t best = INF_H;
        for (int64_t p = 0; p < prev->live.n; p++) if (prev->val[prev->live.a[p]] < best) best = prev->val[prev->live.a[p]];
        out[0] = best >= INF_H ? -1 : best; out[1] = -1; out[2] = -1;
        if (best < INF_H) {
            int64_t bestc = -1;
            for (int64_t p = 0; p < prev->live.n; p++) {
                int64_t c = prev->live.a[p];
                if (prev->val[c] != best) continue;
                int32_t v = g.cell_v[c];
                int64_t j = c - g.base[v];
                if (j == 0 && v != v_s) continue;
                if (bestc < 0 || c < bestc) bestc = c;   /* cell order == (v, j) order */
            }
            out[1] = g.cell_v[bestc]; out[2] = (int32_t)(bestc - g.base[out[1]]);
        }
    }
done:
    if (bk) { for (int32_t b = 0; b <= D; b++) free(bk[b].a); }
    free(bk); free(A.val); free(B.val); free(A.live.a); free(B.live.a);
    graph_free(&g);
    return rc;
}

/* Many reads against one graph, OpenMP over reads (dynamic schedule, in
 * the order given).  caps[r] < 0 selects the dense form for read r.
 * out is 3 ints per read; returns the number of reads that failed. */
int orc_dp_batch(int32_t n, const uint8_t *seq, const int64_t *off, int64_t ne,
                 const int32_t *src, const int32_t *dst,
                 int32_t n_reads, const uint8_t *reads, const int64_t *read_off,
                 const int32_t *v_start, const int32_t *caps, int32_t *out, int32_t n_threads)
{
    int fails = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fails)
#endif
    for (int32_t r = 0; r < n_reads; r++) {
        int32_t o4[4];
        const uint8_t *q = reads + read_off[r];
        int32_t ql = (int32_t)(read_off[r + 1] - read_off[r]);
        int rc = caps[r] < 0 ? orc_dp_dense(n, seq, off, ne, src, dst, q, ql, v_start[r], o4)
                             : orc_dp_capped(n, seq, off, ne, src, dst, q, ql, v_start[r], caps[r], o4);
        if (rc) { fails++; o4[0] = o4[1] = o4[2] = -2; }
        out[3 * r] = o4[0]; out[3 * r + 1] = o4[1]; out[3 * r + 2] = o4[2];
    }
    return fails;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* pairwise edit distance                                               */
/* ------------------------------------------------------------------ */
int64_t orc_ed_global(const uint8_t *a, int64_t na, const uint8_t *b, int64_t nb)
{
    int64_t *row = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb + 1));
    if (!row) return -1;
    for (int64_t j = 0; j <= nb; j++) row[j] = j;
    for (int64_t i = 1; i <= na; i++) {
        int64_t diag = row[0];
        row[0] = i;
        for (int64_t j = 1; j <= nb; j++) {
            int64_t up_ = row[j];
            int64_t x = diag + (up(a[i - 1]) == up(b[j - 1]) ? 0 : 1);
            if (up_ + 1 < x) x = up_ + 1;
            if (row[j - 1] + 1 < x) x = row[j - 1] + 1;
            row[j] = x;
            diag = up_;
        }
    }
    int64_t r = row[nb];
    free(row);
    return r;
}

/* Edit distance restricted to cells with |i-j| <= D; returns -1 when the
 * distance exceeds D (every alignment of cost <= D stays inside the band). */
int64_t orc_ed_banded(const uint8_t *a, int64_t na, const uint8_t *b, int64_t nb, int64_t D)
{
    if (D < 0) return -1;
    int64_t diff = na > nb ? na - nb : nb - na;
    if (diff > D) return -1;
    const int64_t INF = INT64_MAX / 4;
    int64_t W = 2 * D + 1;
    int64_t *prev = (int64_t *)malloc(sizeof(int64_t) * (size_t)W);
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)W);
    if (!prev || !cur) { free(prev); free(cur); return -2; }
    /* slot t of row i holds column j = i - D + t */
    for (int64_t t = 0; t < W; t++) {
        int64_t j = 0 - D + t;
        prev[t] = (j >= 0 && j <= nb) ? j : INF;
    }
    for (int64_t i = 1; i <= na; i++) {
        for (int64_t t = 0; t < W; t++) {
            int64_t j = i - D + t;
            if (j < 0 || j > nb) { cur[t] = INF; continue; }
            int64_t x = INF;
            if (j == 0) x = i;
            else {
                /* (i-1, j-1) is slot t of the previous row */
                if (prev[t] < INF) x = prev[t] + (up(a[i - 1]) == up(b[j - 1]) ? 0 : 1);
                if (t > 0 && cur[t - 1] < INF && cur[t - 1] + 1 < x) x = cur[t - 1] + 1;   /* (i, j-1) */
            }
            /* (i-1, j) is slot t+1 of the previous row */
            if (t + 1 < W && prev[t + 1] < INF && prev[t + 1] + 1 < x) x = prev[t + 1] + 1;
            cur[t] = x;
        }
        int64_t *s = prev; prev = cur; cur = s;
    }
    int64_t tt = nb - na + D;
    int64_t r = (tt >= 0 && tt < W) ? prev[tt] : INF;
    free(prev); free(cur);
    return (r > D || r >= INF) ? -1 : r;
}

/* ------------------------------------------------------------------ */
/* Algorithms 1-4: wavefront driver, extension, expansion, pruning      */
/* ------------------------------------------------------------------ */
/* Graph wavefront set H~ (Section 2.4): a map from diagonal (v,k) to its
 * furthest offset, plus the aligned walk length W~ that Algorithm 4 uses.
 * Entries are never removed, so older offsets stay as the record that the
 * dominance tests of Algorithms 2-3 compare against. */
typedef struct {
    uint64_t key;      /* 0 = empty slot */
    int32_t off, W;
    int32_t round;     /* crossing round that created it in the current score */
    int32_t pending;   /* created by a crossing and not yet extended */
} hent;

typedef struct { hent *t; uint64_t cap, n; } hmap;

static inline uint64_t dkey(int32_t v, int32_t k)
{
    return ((uint64_t)(uint32_t)(v + 1) << 32) | (uint32_t)(k + 0x40000000);
}
static inline uint64_t mix64(uint64_t x)
{
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL; x ^= x >> 33;
    return x;
}
static hent *hm_find(hmap *m, uint64_t key)
{
    uint64_t i = mix64(key) & (m->cap - 1);
    for (;;) {
        if (m->t[i].key == key) return &m->t[i];
        if (m->t[i].key == 0) return NULL;
        i = (i + 1) & (m->cap - 1);
    }
}
static int hm_grow(hmap *m);
static hent *hm_insert(hmap *m, uint64_t key)
{
    if ((m->n + 1) * 2 > m->cap && hm_grow(m)) return NULL;
    uint64_t i = mix64(key) & (m->cap - 1);
    while (m->t[i].key != 0 && m->t[i].key != key) i = (i + 1) & (m->cap - 1);
    if (m->t[i].key == 0) { m->t[i].key = key; m->n++; }
    return &m->t[i];
}
static int hm_grow(hmap *m)
{
    uint64_t nc = m->cap ? m->cap * 2 : 1024;
    hent *nt = (hent *)calloc((size_t)nc, sizeof(hent));
    if (!nt) return -1;
    for (uint64_t i = 0; i < m->cap; i++) {
        if (!m->t[i].key) continue;
        uint64_t j = mix64(m->t[i].key) & (nc - 1);
        while (nt[j].key) j = (j + 1) & (nc - 1);
        nt[j] = m->t[i];
    }
    free(m->t); m->t = nt; m->cap = nc;
    return 0;
}

typedef struct { int32_t *v, *k; int64_t n, cap; } dqueue;
static int dq_push(dqueue *q, int32_t v, int32_t k)
{
    if (q->n == q->cap) {
        int64_t nc = q->cap ? q->cap * 2 : 256;
        int32_t *nv = (int32_t *)realloc(q->v, sizeof(int32_t) * (size_t)nc);
        if (!nv) return -1;
        q->v = nv;
        int32_t *nk = (int32_t *)realloc(q->k, sizeof(int32_t) * (size_t)nc);
        if (!nk) return -1;
        q->k = nk; q->cap = nc;
    }
    q->v[q->n] = v; q->k[q->n] = k; q->n++;
    return 0;
}

/* Options / outputs of orc_gwf.
 *   a_diff      <= 0: exact; > 0: Algorithm 4 between the end test and the
 *               expansion (the paper places it between its d <- d+1 and the
 *               call to the expansion).
 *   max_score   stop with status 1 when d exceeds it (-1: unbounded).
 *   e_free      free end gap in the query: the end test takes any row
 *               i >= |q| - e_free (0: the whole query).
 *   wfree       global form with a free end gap in the walk: the end test
 *               of extension mode restricted to cells of v_e.
 * out[0] = distance (-1 when stopped), out[1..2] = end (v, j), out[3] = status,
 * out[4] = query bases left unaligned.
 * work[0] = sum over scores of |F_s| (entries after extension, before
 * pruning); work[1] = number of diagonals ever created (size of H~);
 * work[2] = crossings admitted.  counts (optional) receives |F_s| for
 * s < counts_cap.  ent (optional) receives five words per entry of every
 * extended wavefront, score by score: (d, v, k, offset, W~), at most
 * ent_cap entries; *ent_n gets the number there were. */
int orc_gwf(int32_t n, const uint8_t *seq, const int64_t *off, int64_t ne,
            const int32_t *src, const int32_t *dst,
            const uint8_t *q, int32_t qlen, int32_t v_s, int32_t j0, int32_t j1, int32_t v_e, int32_t wfree,
            int32_t e_free, int32_t a_diff, int32_t max_score, int32_t *out, int64_t *work, int32_t *counts, int32_t counts_cap,
            int32_t *ent, int64_t ent_cap, int64_t *ent_n)
{
    ograph g;
    if (graph_init(&g, n, seq, off, ne, src, dst, 0)) { graph_free(&g); return -1; }
    if (j1 < 0) j1 = j0;
    if (v_s < 0 || v_s >= n || v_e >= n || j0 < 0 || j1 < j0 || j1 > vlen(&g, v_s) || e_free < 0 ||
        e_free > qlen) {
        graph_free(&g);
        return -1;
    }
    const int32_t i_lo = qlen - e_free;   /* end rows: i_lo .. |q| */
    hmap H = {0, 0, 0};
    dqueue Q = {0}, Qn = {0}, X = {0};
    int rc = 0;
    out[0] = -1; out[1] = -1; out[2] = -1; out[3] = 0; out[4] = 0;
    work[0] = work[1] = work[2] = 0;
    if (ent_n) *ent_n = 0;
    if (hm_grow(&H)) { rc = -1; goto done; }

    /* Algorithm 1: H~_{v_s,0} <- 0; Q <- [(v_s,0)]; d <- 0.  A walk that
     * starts after the first j bases of v_s starts on diagonal -j (the cell
     * (0, v_s, j)) at offset j; a start window j0..j1 puts all of them in
     * the score-0 wavefront. */
    for (int32_t j = j0; j <= j1; j++) {
        hent *e = hm_insert(&H, dkey(v_s, -j));
        if (!e) { rc = -1; goto done; }
        e->off = j; e->W = 0; e->round = 0; e->pending = 0;
        if (dq_push(&Q, v_s, -j)) { rc = -1; goto done; }
    }
    for (int32_t d = 0;; d++) {
        if (max_score >= 0 && d > max_score) { out[3] = 1; break; }
        /* ---- Algorithm 2 (extension).  Q is consumed first-in first-out, so
         * entries created by crossings form rounds: every round-r diagonal
         * is extended before any round-(r+1) one.  A crossing target that was
         * created in the same round by another predecessor takes the larger
         * walk length W. */
        X.n = 0;
        for (int64_t p = 0; p < Q.n; p++) if (dq_push(&X, Q.v[p], Q.k[p])) { rc = -1; goto done; }
        Qn.n = 0;
        for (int64_t p = 0; p < X.n; p++) {
            int32_t v = X.v[p], k = X.k[p];
            hent *e = hm_find(&H, dkey(v, k));
            int32_t j = e->off, i = k + j;
            int32_t L = (int32_t)vlen(&g, v);
            const uint8_t *lab = seq + off[v];
            int32_t l = 0;
            while (i + l < qlen && j + l < L && up(q[i + l]) == up(lab[j + l])) l++;   /* LCP */
            e->off = j + l;
            e->W += l;
            int32_t my_round = e->round;
            e->pending = 0;
            if (dq_push(&Qn, v, k)) { rc = -1; goto done; }
            if (e->off == L) {
                int32_t W = e->W;
                for (int32_t ed = g.out_off[v]; ed < g.out_off[v + 1]; ed++) {
                    int32_t u = g.out_dst[ed], k2 = k + L;
                    hent *t = hm_find(&H, dkey(u, k2));
                    if (!t) {
                        t = hm_insert(&H, dkey(u, k2));
                        if (!t) { rc = -1; goto done; }
                        t->off = 0; t->W = W; t->round = my_round + 1; t->pending = 1;
                        work[2]++;
                        if (dq_push(&X, u, k2)) { rc = -1; goto done; }
                        e = hm_find(&H, dkey(v, k));           /* the table may have moved */
                    } else if (t->pending && t->round == my_round + 1 && W > t->W) {
                        t->W = W;
                    }
                }
            }
        }
        for (int64_t p = 0; p < Qn.n; p++) hm_find(&H, dkey(Qn.v[p], Qn.k[p]))->round = 0;
        work[0] += Qn.n;
        if (counts && d < counts_cap) counts[d] = (int32_t)Qn.n;
        if (ent && ent_n) {
            for (int64_t p = 0; p < Qn.n; p++) {
                if (*ent_n < ent_cap) {
                    const hent *e = hm_find(&H, dkey(Qn.v[p], Qn.k[p]));
                    int32_t *w = ent + 5 * *ent_n;
                    w[0] = d; w[1] = Qn.v[p]; w[2] = Qn.k[p]; w[3] = e->off; w[4] = e->W;
                }
                (*ent_n)++;
            }
        }

        /* ---- end test, global form (Algorithm 1 as printed): the diagonal
         * of the end cell (v_e, |q| - |v_e|) has reached offset |v_e|.  An
         * empty wavefront means v_e cannot be reached (out[3] = 2). */
        if (v_e >= 0 && !wfree) {
            /* with a free end gap, the cell (i, v_e, |v_e|) of the largest
             * i >= |q| - e_free that has been reached */
            int32_t Le = (int32_t)vlen(&g, v_e), hit = -1;
            for (int32_t i = qlen; i >= i_lo && hit < 0; i--) {
                hent *e = hm_find(&H, dkey(v_e, i - Le));
                if (e && e->off == Le) hit = i;
            }
            if (hit >= 0) { out[0] = d; out[1] = v_e; out[2] = Le; out[4] = qlen - hit; break; }
            if (Qn.n == 0) { out[3] = 2; break; }
        }
        /* ---- end test (extension mode, and the global form with a free
         * end gap in the walk): some wavefront cell that can end a walk (in
         * v_e for the latter) has consumed the whole query.  A cell (v, 0)
         * ends a walk only at the start (v_s with offset 0): otherwise it is
         * the copy of a predecessor's last cell. */
        if (v_e < 0 || wfree) {
            /* the largest i >= |q| - e_free over those front cells, then the
             * smallest (v, j) among that row's */
            int32_t imax = -1, bv = -1, bj = -1;
            for (int64_t p = 0; p < Qn.n; p++) {
                int32_t v = Qn.v[p];
                hent *e = hm_find(&H, dkey(v, Qn.k[p]));
                int32_t i = Qn.k[p] + e->off;
                if (v_e >= 0 && v != v_e) continue;
                if (e->off == 0 && !(v == v_s && j0 == 0)) continue;
                if (i >= i_lo && i > imax) imax = i;
            }
            for (int64_t p = 0; p < Qn.n && imax >= 0; p++) {
                int32_t v = Qn.v[p], k = Qn.k[p];
                hent *e = hm_find(&H, dkey(v, k));
                if (k + e->off != imax) continue;
                if (v_e >= 0 && v != v_e) continue;
                if (e->off == 0 && !(v == v_s && j0 == 0)) continue;
                if (bv < 0 || v < bv || (v == bv && e->off < bj)) { bv = v; bj = e->off; }
            }
            if (imax >= 0) { out[0] = d; out[1] = bv; out[2] = bj; out[4] = qlen - imax; break; }
            if (v_e >= 0 && Qn.n == 0) { out[3] = 2; break; }
        }

        /* ---- Algorithm 4 (pruning) on the extended wavefront */
        if (a_diff > 0) {
            int64_t amax = 0;
            for (int64_t p = 0; p < Qn.n; p++) {
                hent *e = hm_find(&H, dkey(Qn.v[p], Qn.k[p]));
                int64_t a = (int64_t)Qn.k[p] + e->off + e->W;
                if (a > amax) amax = a;
            }
            if (amax > a_diff) {
                int64_t w = 0;
                for (int64_t p = 0; p < Qn.n; p++) {
                    hent *e = hm_find(&H, dkey(Qn.v[p], Qn.k[p]));
                    int64_t a = (int64_t)Qn.k[p] + e->off + e->W;
                    if (amax - a < a_diff) { Qn.v[w] = Qn.v[p]; Qn.k[w] = Qn.k[p]; w++; }
                }
                Qn.n = w;   /* dropped diagonals keep their offsets in H~ */
            }
        }

        /* ---- Algorithm 3 (expansion) into the (d+1)-wave.  Each candidate
         * (insertion, deletion, mismatch) is kept per diagonal as the largest
         * offset, ties broken by the larger W; it is admitted when the
         * diagonal has no offset in H~ yet or its offset there is smaller. */
        {
            hmap Hn = {0, 0, 0};
            dqueue Cand = {0};
            if (hm_grow(&Hn)) { rc = -1; goto done; }
            for (int64_t p = 0; p < Qn.n; p++) {
                int32_t v = Qn.v[p], k = Qn.k[p];
                hent *e = hm_find(&H, dkey(v, k));
                int32_t o = e->off, W = e->W, i = k + o, L = (int32_t)vlen(&g, v);
                int32_t cv[3], ck[3], co[3], cw[3], nc = 0;
                if (i < qlen) { cv[nc] = v; ck[nc] = k + 1; co[nc] = o; cw[nc] = W; nc++; }             /* insertion */
                if (o < L) { cv[nc] = v; ck[nc] = k - 1; co[nc] = o + 1; cw[nc] = W + 1; nc++; }       /* deletion */
                if (i < qlen && o < L) { cv[nc] = v; ck[nc] = k; co[nc] = o + 1; cw[nc] = W + 1; nc++; } /* mismatch */
                for (int c = 0; c < nc; c++) {
                    hent *old = hm_find(&H, dkey(cv[c], ck[c]));
                    if (old && old->off >= co[c]) continue;        /* dominated */
                    hent *t = hm_find(&Hn, dkey(cv[c], ck[c]));
                    if (!t) {
                        t = hm_insert(&Hn, dkey(cv[c], ck[c]));
                        if (!t) { rc = -1; free(Hn.t); free(Cand.v); free(Cand.k); goto done; }
                        t->off = co[c]; t->W = cw[c];
                        dq_push(&Cand, cv[c], ck[c]);
                    } else if (co[c] > t->off || (co[c] == t->off && cw[c] > t->W)) {
                        t->off = co[c]; t->W = cw[c];
                    }
                }
            }
            Q.n = 0;
            for (int64_t p = 0; p < Cand.n; p++) {
                hent *t = hm_find(&Hn, dkey(Cand.v[p], Cand.k[p]));
                hent *e = hm_insert(&H, dkey(Cand.v[p], Cand.k[p]));
                if (!e) { rc = -1; break; }
                e->off = t->off; e->W = t->W; e->round = 0; e->pending = 0;
                dq_push(&Q, Cand.v[p], Cand.k[p]);
            }
            free(Hn.t); free(Cand.v); free(Cand.k);
            if (rc) goto done;
        }
    }
    work[1] = (int64_t)H.n;
done:
    free(H.t); free(Q.v); free(Q.k); free(Qn.v); free(Qn.k); free(X.v); free(X.k);
    graph_free(&g);
    return rc;
}
