// gwfa_labels.cpp -- training labels for the learned pruning network (host).
//
// A wavefront entry of score s whose front cell is (i, v, off) lies on an
// optimal alignment exactly when s + R(i, v, off) = d*, where R is the cost
// of the best completion of the alignment from that cell to the end of the
// query (the end is free anywhere in the graph, as in the extension form of
// Eq. 1).  R obeys Eq. 1 read backwards:
//   R(|q|, v, j) = 0;
//   R(i, v, j)   = min( R(i+1, v, j) + 1,                      insertion
//                       R(i, v, j+1) + 1             (j < |v|), deletion
//                       R(i+1, v, j+1) + [q_{i+1} != v_{j+1}] (j < |v|) )
//   R(i, v, |v|) also takes min over out-edges (v,u) of R(i, u, 0) at cost 0;
// and d* = R(0, v_s, 0).
//
// Rows are computed from i = |q| down to 0, two rows in memory.  Inside a row
// the deletion and edge terms form a shortest-path problem; it is solved on
// the vertex level: with A_u = min over j < |u| of (T(u,j) + j), where T is
// the value before the in-row terms, the value X_v = R(i, v, |v|) satisfies
//   X_v = min( T(v,|v|), min over (v,u) of min(A_u, X_u + |u|) ),
// a single-source-free shortest path with positive edge weights |u| >= 1,
// settled by Dijkstra's algorithm over predecessor lists; each vertex's
// interior cells then follow in one backward scan.
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <functional>
#include <queue>
#include <thread>
#include <utility>
#include <vector>

#include "gwfa.h"

namespace {

constexpr int32_t INF = 0x3fffffff;

inline int code_of(uint8_t c) {
    switch (c & 0xdf) {
        case 'A': return 0;
        case 'C': return 1;
        case 'G': return 2;
        case 'T': return 3;
        default: return -1;
    }
}

struct LabelGraph {
    int32_t n_vtx = 0;
    std::vector<int64_t> cell0;      // first cell of each vertex: cells (v,0..|v|)
    std::vector<int32_t> len;
    std::vector<int8_t> base;        // codes of all labels, concatenated
    std::vector<int64_t> boff;
    std::vector<int32_t> out_off, out_dst, in_off, in_src;
    int64_t n_cells = 0;
};

void reverse_costs(const LabelGraph& G, const int8_t* q, int32_t qlen, int32_t v_s,
                   const std::vector<int64_t>& ents, const int32_t* ent_i, const int32_t* ent_v,
                   const int32_t* ent_off, int32_t* cost_out, int32_t* dist_out) {
    const int32_t V = G.n_vtx;
    std::vector<int32_t> nxt(G.n_cells, 0), cur(G.n_cells, 0), A(V), X(V);
    std::vector<char> done(V);
    // entries bucketed by row
    std::vector<int64_t> row_first(qlen + 2, 0), order(ents.size());
    for (int64_t e : ents) row_first[ent_i[e] + 1]++;
    for (int32_t i = 0; i <= qlen; ++i) row_first[i + 1] += row_first[i];
    {
        std::vector<int64_t> fill(row_first.begin(), row_first.end() - 1);
        for (int64_t e : ents) order[fill[ent_i[e]]++] = e;
    }
    auto settle_row = [&](int32_t i, const std::vector<int32_t>& row) {
        for (int64_t t = row_first[i]; t < row_first[i + 1]; ++t) {
            const int64_t e = order[t];
            cost_out[e] = row[G.cell0[ent_v[e]] + ent_off[e]];
        }
    };
    // row |q|: every cell is an end
    settle_row(qlen, nxt);
    using Item = std::pair<int32_t, int32_t>;
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    for (int32_t i = qlen - 1; i >= 0; --i) {
        const int c = q[i];
        // values before the in-row terms; A_v
        for (int32_t v = 0; v < V; ++v) {
            const int64_t c0 = G.cell0[v];
            const int32_t L = G.len[v];
            const int8_t* lab = &G.base[G.boff[v]];
            int32_t a = INF;
            for (int32_t j = 0; j < L; ++j) {
                const int32_t t = std::min(nxt[c0 + j] + 1, nxt[c0 + j + 1] + (lab[j] != c ? 1 : 0));
                cur[c0 + j] = t;
                a = std::min(a, t + j);
            }
            cur[c0 + L] = nxt[c0 + L] + 1;
            A[v] = a;
        }
        // X_v by Dijkstra from the tentative values
        for (int32_t v = 0; v < V; ++v) {
            int32_t x = cur[G.cell0[v] + G.len[v]];
            for (int32_t e = G.out_off[v]; e < G.out_off[v + 1]; ++e) x = std::min(x, A[G.out_dst[e]]);
            X[v] = x;
            done[v] = 0;
            heap.push({x, v});
        }
        while (!heap.empty()) {
            const Item it = heap.top();
            heap.pop();
            const int32_t u = it.second;
            if (done[u] || it.first != X[u]) continue;
            done[u] = 1;
            const int32_t through = X[u] + G.len[u];
            for (int32_t e = G.in_off[u]; e < G.in_off[u + 1]; ++e) {
                const int32_t v = G.in_src[e];
                if (!done[v] && through < X[v]) {
                    X[v] = through;
                    heap.push({through, v});
                }
            }
        }
        // interior cells, backwards along each vertex
        for (int32_t v = 0; v < V; ++v) {
            const int64_t c0 = G.cell0[v];
            const int32_t L = G.len[v];
            cur[c0 + L] = X[v];
            for (int32_t j = L - 1; j >= 0; --j) cur[c0 + j] = std::min(cur[c0 + j], cur[c0 + j + 1] + 1);
        }
        settle_row(i, cur);
        std::swap(cur, nxt);
    }
    *dist_out = nxt[G.cell0[v_s]];   // row 0 after the final swap
}

}  // namespace

extern "C" int gwfa_label_entries(int32_t n_vtx, const uint8_t* seq, const int64_t* seq_off, int64_t n_edge,
                                  const int32_t* edge_src, const int32_t* edge_dst, int32_t n_reads,
                                  const uint8_t* reads, const int64_t* read_off, const int32_t* v_start,
                                  int64_t n_ent, const int32_t* ent_read, const int32_t* ent_score,
                                  const int32_t* ent_i, const int32_t* ent_v, const int32_t* ent_off,
                                  int32_t* out_cost, uint8_t* out_label, int32_t* out_dist, int32_t n_threads) {
    if (n_vtx <= 0 || !seq_off || n_edge < 0 || n_reads < 0 || n_ent < 0) return GWFA_ERR_ARG;
    if (n_edge > 0 && (!edge_src || !edge_dst)) return GWFA_ERR_ARG;
    if (n_reads > 0 && (!read_off || !v_start || !out_dist)) return GWFA_ERR_ARG;
    if (n_ent > 0 && (!ent_read || !ent_score || !ent_i || !ent_v || !ent_off || !out_cost)) return GWFA_ERR_ARG;
    if (seq_off[0] != 0) return GWFA_ERR_ARG;
    LabelGraph G;
    G.n_vtx = n_vtx;
    G.cell0.resize(n_vtx);
    G.len.resize(n_vtx);
    G.boff.resize(n_vtx);
    for (int32_t v = 0; v < n_vtx; ++v) {
        const int64_t L = seq_off[v + 1] - seq_off[v];
        if (L < 0) return GWFA_ERR_ARG;
        if (L == 0) return GWFA_ERR_EMPTY_LABEL;
        if (L > (1 << 30)) return GWFA_ERR_ARG;
        G.len[v] = (int32_t)L;
        G.boff[v] = seq_off[v];
        G.cell0[v] = G.n_cells;
        G.n_cells += L + 1;
    }
    const int64_t bases = seq_off[n_vtx];
    if (bases > 0 && !seq) return GWFA_ERR_ARG;
    G.base.resize(bases);
    for (int64_t b = 0; b < bases; ++b) {
        const int c = code_of(seq[b]);
        if (c < 0) return GWFA_ERR_ALPHABET;
        G.base[b] = (int8_t)c;
    }
    for (int64_t e = 0; e < n_edge; ++e)
        if (edge_src[e] < 0 || edge_src[e] >= n_vtx || edge_dst[e] < 0 || edge_dst[e] >= n_vtx) return GWFA_ERR_VERTEX;
    G.out_off.assign(n_vtx + 1, 0);
    G.in_off.assign(n_vtx + 1, 0);
    for (int64_t e = 0; e < n_edge; ++e) {
        G.out_off[edge_src[e] + 1]++;
        G.in_off[edge_dst[e] + 1]++;
    }
    for (int32_t v = 0; v < n_vtx; ++v) {
        G.out_off[v + 1] += G.out_off[v];
        G.in_off[v + 1] += G.in_off[v];
    }
    G.out_dst.resize(std::max<int64_t>(n_edge, 1));
    G.in_src.resize(std::max<int64_t>(n_edge, 1));
    {
        std::vector<int32_t> fo(G.out_off.begin(), G.out_off.end() - 1), fi(G.in_off.begin(), G.in_off.end() - 1);
        for (int64_t e = 0; e < n_edge; ++e) {
            G.out_dst[fo[edge_src[e]]++] = edge_dst[e];
            G.in_src[fi[edge_dst[e]]++] = edge_src[e];
        }
    }
    if (n_reads == 0) return n_ent == 0 ? GWFA_OK : GWFA_ERR_ARG;
    if (read_off[0] != 0) return GWFA_ERR_ARG;
    for (int32_t r = 0; r < n_reads; ++r) {
        if (read_off[r + 1] < read_off[r] || read_off[r + 1] - read_off[r] > (1 << 30)) return GWFA_ERR_ARG;
        if (v_start[r] < 0 || v_start[r] >= n_vtx) return GWFA_ERR_VERTEX;
    }
    const int64_t qb = read_off[n_reads];
    if (qb > 0 && !reads) return GWFA_ERR_ARG;
    std::vector<int8_t> qc(qb);
    for (int64_t b = 0; b < qb; ++b) {
        const int c = code_of(reads[b]);
        if (c < 0) return GWFA_ERR_ALPHABET;
        qc[b] = (int8_t)c;
    }
    // entries grouped by read, validated
    std::vector<int64_t> first(n_reads + 1, 0), byread(n_ent);
    for (int64_t e = 0; e < n_ent; ++e) {
        const int32_t r = ent_read[e];
        if (r < 0 || r >= n_reads) return GWFA_ERR_ARG;
        const int64_t qlen = read_off[r + 1] - read_off[r];
        if (ent_i[e] < 0 || ent_i[e] > qlen || ent_v[e] < 0 || ent_v[e] >= n_vtx || ent_off[e] < 0 ||
            ent_off[e] > G.len[ent_v[e]] || ent_score[e] < 0)
            return GWFA_ERR_ARG;
        first[r + 1]++;
    }
    for (int32_t r = 0; r < n_reads; ++r) first[r + 1] += first[r];
    {
        std::vector<int64_t> fill(first.begin(), first.end() - 1);
        for (int64_t e = 0; e < n_ent; ++e) byread[fill[ent_read[e]]++] = e;
    }
    // longest reads first over a pool of threads
    std::vector<int32_t> ord(n_reads);
    for (int32_t r = 0; r < n_reads; ++r) ord[r] = r;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        return read_off[a + 1] - read_off[a] > read_off[b + 1] - read_off[b];
    });
    int nt = n_threads > 0 ? n_threads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = std::min<int>(nt, std::max(1, n_reads));
    std::atomic<int32_t> next{0};
    auto work = [&]() {
        std::vector<int64_t> ents;
        for (;;) {
            const int32_t t = next.fetch_add(1);
            if (t >= n_reads) break;
            const int32_t r = ord[t];
            ents.assign(byread.begin() + first[r], byread.begin() + first[r + 1]);
            reverse_costs(G, qc.data() + read_off[r], (int32_t)(read_off[r + 1] - read_off[r]), v_start[r], ents,
                          ent_i, ent_v, ent_off, out_cost, &out_dist[r]);
        }
    };
    std::vector<std::thread> pool;
    for (int k = 1; k < nt; ++k) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
    if (out_label)
        for (int64_t e = 0; e < n_ent; ++e)
            out_label[e] = (ent_score[e] + out_cost[e] == out_dist[ent_read[e]]) ? 1 : 0;
    return GWFA_OK;
}
