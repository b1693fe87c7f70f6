/*
 * labels.c -- reverse form of Eq. 1 (TEST INFRASTRUCTURE ONLY; see oracle.c).
 *
 * R_{i,v,j} is the least cost of consuming the rest of the query,
 * q[i+1..|q|], starting from DP cell (i,v,j) in extension mode (the end is
 * free).  It mirrors the four cases of Eq. 1 read backwards:
 *   R_{|q|,v,j} = 0
 *   R_{i,v,j}   = min( R_{i+1,v,j} + 1                       (consume q[i+1])
 *                      R_{i,v,j+1} + 1,            j < |v|    (consume v[j+1])
 *                      R_{i+1,v,j+1} + Delta,      j < |v|    (align both)
 *                      R_{i,u,0},      j = |v|, (v,u) in E )  (cross an edge)
 * A wavefront entry at score s whose front cell is (i,v,j) lies on an
 * optimal alignment exactly when s + R_{i,v,j} = d*.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define INF_R (INT32_MAX / 4)

static inline uint8_t up_(uint8_t c) { return (c >= 'a' && c <= 'z') ? (uint8_t)(c - 32) : c; }

/* For each entry e: out_cost[e] = R_{ent_i[e], ent_v[e], ent_off[e]}.
 * out_dstar[0] = R_{0,v_s,0} (= d*).  Returns 0, or -1 on failure. */
int orc_rev_labels(int32_t n, const uint8_t *seq, const int64_t *off, int64_t ne,
                   const int32_t *src, const int32_t *dst,
                   const uint8_t *q, int32_t qlen, int32_t v_s,
                   const int32_t *ent_i, const int32_t *ent_v, const int32_t *ent_off,
                   int32_t *out_cost, int64_t nent, int32_t *out_dstar)
{
    int64_t *base = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *oo = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *od = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    if (!base || !oo || !od) { free(base); free(oo); free(od); return -1; }
    for (int32_t v = 0; v <= n; v++) base[v] = off[v] + v;
    int64_t ncell = base[n];
    for (int64_t e = 0; e < ne; e++) oo[src[e] + 1]++;
    for (int32_t v = 0; v < n; v++) oo[v + 1] += oo[v];
    {
        int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
        if (!fill) { free(base); free(oo); free(od); return -1; }
        memcpy(fill, oo, sizeof(int32_t) * (size_t)(n + 1));
        for (int64_t e = 0; e < ne; e++) od[fill[src[e]]++] = dst[e];
        free(fill);
    }
    int32_t *R = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncell * (size_t)(qlen + 1));
    if (!R) { free(base); free(oo); free(od); return -1; }
    int rc = 0;
    for (int32_t i = qlen; i >= 0; i--) {
        int32_t *row = R + (size_t)i * (size_t)ncell;
        if (i == qlen) {
            for (int64_t c = 0; c < ncell; c++) row[c] = 0;
            continue;
        }
        const int32_t *nx = R + (size_t)(i + 1) * (size_t)ncell;
        uint8_t qi = up_(q[i]);   /* q[i+1] in 1-based terms */
        for (int32_t v = 0; v < n; v++) {
            int64_t c0 = base[v], L = off[v + 1] - off[v];
            for (int64_t j = 0; j <= L; j++) {
                int32_t h = nx[c0 + j] + 1;
                if (j < L) {
                    int32_t x = nx[c0 + j + 1] + (qi == up_(seq[off[v] + j]) ? 0 : 1);
                    if (x < h) h = x;
                }
                row[c0 + j] = h;
            }
        }
        /* in-row terms (consume a base of v, cross an edge), swept in
         * reverse vertex order until nothing changes */
        int changed, sweeps = 0;
        do {
            changed = 0;
            if (++sweeps > n + 2) { rc = -1; break; }
            for (int32_t v = n - 1; v >= 0; v--) {
                int64_t c0 = base[v], L = off[v + 1] - off[v];
                for (int32_t e = oo[v]; e < oo[v + 1]; e++) {
                    int32_t x = row[base[od[e]]];
                    if (x < row[c0 + L]) { row[c0 + L] = x; changed = 1; }
                }
                for (int64_t j = L - 1; j >= 0; j--)
                    if (row[c0 + j + 1] + 1 < row[c0 + j]) { row[c0 + j] = row[c0 + j + 1] + 1; changed = 1; }
            }
        } while (changed);
        if (rc) break;
    }
    if (rc == 0) {
        out_dstar[0] = R[base[v_s]];
        for (int64_t e = 0; e < nent; e++) {
            int32_t i = ent_i[e], v = ent_v[e], j = ent_off[e];
            if (i < 0 || i > qlen || v < 0 || v >= n || j < 0 || j > off[v + 1] - off[v]) { out_cost[e] = -1; continue; }
            out_cost[e] = R[(size_t)i * (size_t)ncell + (size_t)(base[v] + j)];
        }
    }
    free(R); free(base); free(oo); free(od);
    return rc;
}
