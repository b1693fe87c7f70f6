// gwfa_kernels.hip -- device code of the graph wavefront alignment library
// for AMD CDNA4 (gfx950).
//
// One persistent workgroup aligns one query at a time, taking queries from a
// device work queue.  Per score s it runs the paper's loop (Section 2.4):
//   EXTEND  (Algorithm 2): slide every diagonal of F_s along its vertex by the
//           exact-match run (2-bit packed XOR + count-leading-zeros, 32 bases
//           per step); a diagonal reaching the end of vertex v creates
//           (u, k+|v|) at offset 0 on every out-edge (v,u) not seen before,
//           at the same score, and those are extended in further rounds;
//   END     (extension mode): stop at the first score where some cell of the
//           wavefront has consumed the whole query;
//   PRUNE   (Algorithm 4, optional) or the learned keep/drop network;
//   EXPAND  (Algorithm 3): insertion / deletion / mismatch candidates of
//           every diagonal, merged per diagonal, admitted when they beat the
//           diagonal's record.
//
// Per-query state lives in an HBM arena owned by the workgroup:
//   * diagonal records (the paper's wavefront set H~, never cleared while a
//     query runs): pages of 32 consecutive diagonals (v, 32p .. 32p+31),
//     found through an open-addressing page directory keyed (v, p).  A page
//     slot holds the furthest offset, the score stamp of the last time the
//     diagonal was in a wavefront, and (walk length W, trace index t);
//   * the wavefront F_s as a list of entries (v, k, off, W, t, page);
//   * the crossing candidates of the current round;
//   * the traceback array T and its de-duplication map M (Algorithm 5).
//
// EXPAND is owner-computes: the output diagonal k' of vertex v is produced by
// the present source with the smallest k among k'-1, k', k'+1 (present =
// stamped with the current score), which gathers all three sources from the
// page, so no atomics are needed and the result (largest offset, ties to the
// larger W) does not depend on scheduling.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gwfa_internal.h"

namespace gwfa_dev {

typedef unsigned long long ull;

constexpr int PAGE = 32;
constexpr int32_t ST_EMPTY = -1;
constexpr int32_t ST_CLAIM = -2;
constexpr int32_t ST_PRUNED = 0x40000000;

constexpr int F_GROW = 1;   // directory / trace capacity exceeded: restart bigger
constexpr int F_LIST = 2;   // list or candidate capacity exceeded: give up (re-run on a larger tier)

struct Page {
    int32_t off[PAGE];
    int32_t stamp[PAGE];
    ull wt[PAGE];   // (W << 32) | (t + 1)
};
static_assert(sizeof(Page) == 512, "page layout");

__device__ __forceinline__ ull pack_wt(int32_t W, int32_t t) {
    return ((ull)(uint32_t)W << 32) | (ull)(uint32_t)(t + 1);
}
__device__ __forceinline__ int32_t wt_W(ull x) { return (int32_t)(x >> 32); }
__device__ __forceinline__ int32_t wt_t(ull x) { return (int32_t)(uint32_t)(x & 0xffffffffull) - 1; }

__device__ __forceinline__ ull dkey(int32_t v, int32_t kp) {
    return ((ull)(uint32_t)(v + 1) << 32) | (ull)(uint32_t)(kp + 0x40000000);
}
__device__ __forceinline__ uint32_t dhash(ull key) {
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 32);
}

// 32 bases starting at base index p of a 2-bit MSB-first packed store.
__device__ __forceinline__ ull win32(const ull* __restrict__ w, int64_t p) {
    const int64_t wi = p >> 5;
    const int sh = (int)(p & 31) * 2;
    const ull a = w[wi];
    const ull b = w[wi + 1];
    return (a << sh) | ((b >> 1) >> (63 - sh));
}

// LCP of q[qp ...] and segment[sp ...], at most lim bases.
__device__ __forceinline__ int32_t lcp(const ull* __restrict__ qw, int64_t qp, const ull* __restrict__ sw,
                                       int64_t sp, int32_t lim, uint32_t& chunks) {
    int32_t l = 0;
    while (l < lim) {
        const ull x = win32(qw, qp + l) ^ win32(sw, sp + l);
        const int32_t m = x ? (int32_t)(__clzll((long long)x) >> 1) : 32;
        ++chunks;
        if (m >= lim - l) { l = lim; break; }
        l += m;
        if (m < 32) break;
    }
    return l;
}

__device__ int dir_find(const ull* __restrict__ dir, uint32_t mask, ull key) {
    uint32_t h = dhash(key) & mask;
    for (uint32_t p = 0; p <= mask; ++p) {
        const ull c = dir[h];
        if (c == key) return (int)h;
        if (c == 0) return -1;
        h = (h + 1) & mask;
    }
    return -1;
}

__device__ int dir_insert(ull* dir, uint32_t mask, ull key, bool& inserted) {
    uint32_t h = dhash(key) & mask;
    inserted = false;
    for (uint32_t p = 0; p <= mask; ++p) {
        const ull c = __hip_atomic_load(&dir[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (c == key) return (int)h;
        if (c == 0) {
            const ull old = atomicCAS(&dir[h], 0ull, key);
            if (old == 0) { inserted = true; return (int)h; }
            if (old == key) return (int)h;
        }
        h = (h + 1) & mask;
    }
    return -1;
}

__device__ __forceinline__ void page_init(Page* pg) {
    int4* s = reinterpret_cast<int4*>(pg->stamp);
#pragma unroll
    for (int i = 0; i < PAGE / 4; ++i) s[i] = make_int4(ST_EMPTY, ST_EMPTY, ST_EMPTY, ST_EMPTY);
    int4* w = reinterpret_cast<int4*>(pg->wt);
#pragma unroll
    for (int i = 0; i < PAGE / 2; ++i) w[i] = make_int4(0, 0, 0, 0);
}

// Exclusive prefix sum of x over the 64 lanes of the wave, plus the total.
__device__ __forceinline__ int wave_excl_scan(int x, int& total) {
    const int lane = __lane_id();
    int incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    total = __shfl(incl, 63, 64);
    return incl - x;
}

// Reserves cnt consecutive slots from an LDS counter for every lane of the
// wave (one atomic per wave).  Must be reached by all lanes of the wave.
__device__ __forceinline__ int wave_alloc(int cnt, int* counter) {
    int total;
    const int ex = wave_excl_scan(cnt, total);
    int base = 0;
    if (__lane_id() == 0 && total > 0) base = atomicAdd(counter, total);
    base = __shfl(base, 0, 64);
    return base + ex;
}

struct Lists {
    int32_t *v, *k, *o, *w, *t, *d;
};

// Reads a shared word that other threads may update in the phase that just
// ended, so that every thread takes the same decision: barrier, read,
// barrier (nobody can write it again before everybody has read it).
__device__ __forceinline__ int read_uniform(const int& x) {
    __syncthreads();
    const int v = *(const volatile int*)&x;
    __syncthreads();
    return v;
}

struct Shared {
    int32_t read;
    int32_t n[2];
    int32_t ncand;
    int32_t dirn;
    int32_t tn;
    int32_t flags;
    int32_t found;
    int32_t amax;
    int32_t tend;
    int32_t dropped;
    ull endkey;
    ull chunks;
    ull cross;
    ull adm;
    ull mlp;
};

template <int BLOCK>
__device__ void align_read(const KArgs& A, char* __restrict__ arena, int r, Shared& S) {
    const int tid = threadIdx.x;
    const int64_t q0 = A.rd_off[r];
    const int32_t qlen = (int32_t)(A.rd_off[r + 1] - q0);
    const int32_t vs = A.v_start[r];
    gwfa_result* out = A.res + r;
    if (vs < 0 || vs >= A.n_vtx) {
        if (tid == 0) {
            out->dist = -1; out->end_v = -1; out->end_off = -1; out->status = GWFA_ST_BAD_INPUT;
            out->path_off = -1; out->path_len = 0; out->n_scores = 0; out->work = 0;
        }
        return;
    }
    const ull* __restrict__ seg = A.seg;
    const int64_t* __restrict__ seg_off = A.seg_off;
    const int32_t* __restrict__ out_off = A.out_off;
    const int32_t* __restrict__ out_dst = A.out_dst;
    const ull* __restrict__ rd = A.rd;

    ull* dir = reinterpret_cast<ull*>(arena + A.o_dir);
    Page* pages = reinterpret_cast<Page*>(arena + A.o_pages);
    ull* mkey = reinterpret_cast<ull*>(arena + A.o_mkey);
    int32_t* mval = reinterpret_cast<int32_t*>(arena + A.o_mval);
    int32_t* Tv = reinterpret_cast<int32_t*>(arena + A.o_tv);
    int32_t* Tt = reinterpret_cast<int32_t*>(arena + A.o_tt);
    Lists L[2];
    {
        int32_t* base = reinterpret_cast<int32_t*>(arena + A.o_lists);
        const int64_t c = A.list_cap;
        for (int j = 0; j < 2; ++j) {
            int32_t* p = base + (int64_t)j * 6 * c;
            L[j].v = p; L[j].k = p + c; L[j].o = p + 2 * c; L[j].w = p + 3 * c; L[j].t = p + 4 * c; L[j].d = p + 5 * c;
        }
    }
    int32_t* cbase = reinterpret_cast<int32_t*>(arena + A.o_cand);
    const int64_t cc = A.cand_cap;
    int32_t *cu = cbase, *ck = cbase + cc, *cW = cbase + 2 * cc, *ct = cbase + 3 * cc, *cd = cbase + 4 * cc;

    const bool tb = A.traceback != 0;
    // initial directory size: dir_factor slots per 32 query bases
    int cap_log2 = 8;
    {
        const int64_t want = ((int64_t)qlen / 32 + 1) * A.dir_factor;
        while (cap_log2 < A.dir_log2_max && ((int64_t)1 << cap_log2) < want) ++cap_log2;
    }
    int status = -1;
    int32_t s = 0, b = 0;
    int64_t work = 0;
    for (;;) {  // attempts with growing directory
        const uint32_t mask = (1u << cap_log2) - 1;
        const int32_t tcap = (int32_t)((mask + 1) >> 1);
        for (uint32_t i = tid; i <= mask; i += BLOCK) {
            dir[i] = 0;
            if (tb) mkey[i] = 0;
        }
        if (tid == 0) {
            S.n[0] = S.n[1] = 0; S.ncand = 0; S.dirn = 0; S.tn = 0; S.flags = 0;
            S.chunks = 0; S.cross = 0; S.adm = 0; S.mlp = 0; S.dropped = 0;
        }
        __syncthreads();
        if (tid == 0) {
            bool ins;
            const int ds = dir_insert(dir, mask, dkey(vs, 0), ins);
            page_init(&pages[ds]);
            L[0].v[0] = vs; L[0].k[0] = 0; L[0].o[0] = 0; L[0].w[0] = 0; L[0].t[0] = 0; L[0].d[0] = ds;
            S.n[0] = 1; S.dirn = 1;
            if (tb) { Tv[0] = vs; Tt[0] = -1; S.tn = 1; }   // Algorithm 5 on the start vertex
        }
        __syncthreads();
        b = 0; s = 0; work = 0; status = -1;
        bool restart = false;
        int rflags = 0;
        for (;; ++s) {
            // ================= EXTEND (Algorithm 2) =================
            if (tid == 0) { S.found = 0; S.endkey = ~0ull; S.amax = 0; S.ncand = 0; }
            __syncthreads();
            int32_t lo = 0, hi = S.n[b];
            uint32_t chunks = 0;
            for (int round = 0;; ++round) {
                if (round > 0) {
                    // crossing targets admitted last round: take (W, t) from
                    // the slot, where every crossing predecessor of this
                    // round left its max (Algorithm 5 pushes (u, t)).
                    for (int32_t idx = lo + tid; idx < hi; idx += BLOCK) {
                        const int32_t ds = L[b].d[idx], k = L[b].k[idx];
                        const ull x = pages[ds].wt[k & 31];
                        L[b].w[idx] = wt_W(x);
                        const int32_t tp = wt_t(x);
                        L[b].t[idx] = tp;
                        if (tb) {
                            const int32_t v = L[b].v[idx];
                            bool ins;
                            const int ms = dir_insert(mkey, mask, dkey(v, tp), ins);
                            if (ms < 0) {
                                atomicOr(&S.flags, F_GROW);
                            } else if (ins) {
                                const int ti = atomicAdd(&S.tn, 1);
                                if (ti < tcap) { Tv[ti] = v; Tt[ti] = tp; mval[ms] = ti; }
                                else atomicOr(&S.flags, F_GROW);
                            }
                        }
                    }
                    if (tb) {
                        const int f = read_uniform(S.flags);
                        if (f) { rflags = f; restart = true; break; }
                        for (int32_t idx = lo + tid; idx < hi; idx += BLOCK) {
                            const int ms = dir_find(mkey, mask, dkey(L[b].v[idx], L[b].t[idx]));
                            L[b].t[idx] = ms >= 0 ? mval[ms] : -1;
                        }
                    }
                }
                for (int32_t base = lo; base < hi; base += BLOCK) {
                    const int32_t idx = base + tid;
                    int ncand = 0;
                    int32_t e0 = 0, k = 0, Lv = 0, W = 0, t = 0;
                    if (idx < hi) {
                        const int32_t v = L[b].v[idx];
                        k = L[b].k[idx];
                        int32_t o = L[b].o[idx];
                        W = L[b].w[idx];
                        t = L[b].t[idx];
                        const int32_t ds = L[b].d[idx];
                        const int64_t sb = seg_off[v];
                        Lv = (int32_t)(seg_off[v + 1] - sb);
                        int32_t i = k + o;
                        const int32_t lim = min(qlen - i, Lv - o);
                        const int32_t l = lcp(rd, q0 + i, seg, sb + o, lim, chunks);
                        o += l; W += l; i += l;
                        Page* pg = &pages[ds];
                        const int sl = k & 31;
                        pg->off[sl] = o;
                        pg->stamp[sl] = s;
                        pg->wt[sl] = pack_wt(W, t);
                        L[b].o[idx] = o;
                        L[b].w[idx] = W;
                        if (i == qlen) {
                            S.found = 1;
                            if (o >= 1 || v == vs) atomicMin(&S.endkey, ((ull)(uint32_t)v << 32) | (uint32_t)o);
                        }
                        if (A.prune == GWFA_PRUNE_HEURISTIC || A.prune == GWFA_PRUNE_LEARNED) atomicMax(&S.amax, i + W);
                        if (o == Lv) { e0 = out_off[v]; ncand = out_off[v + 1] - e0; }
                    }
                    const int pos = wave_alloc(ncand, &S.ncand);
                    for (int e = 0; e < ncand; ++e) {
                        const int c = pos + e;
                        if (c < A.cand_cap) {
                            cu[c] = out_dst[e0 + e]; ck[c] = k + Lv; cW[c] = W; ct[c] = t;
                        } else {
                            atomicOr(&S.flags, F_LIST);
                        }
                    }
                }
                __syncthreads();
                const int32_t nc = S.ncand;
                {
                    const int f = read_uniform(S.flags);
                    if (f) { rflags = f; restart = true; break; }
                }
                if (nc == 0) break;
                // (a) pages for the crossing targets
                for (int32_t c = tid; c < nc; c += BLOCK) {
                    bool ins;
                    const int ds = dir_insert(dir, mask, dkey(cu[c], ck[c] >> 5), ins);
                    if (ds < 0) atomicOr(&S.flags, F_GROW);
                    else if (ins) { page_init(&pages[ds]); atomicAdd(&S.dirn, 1); }
                    cd[c] = ds;
                }
                {
                    const int f = read_uniform(S.flags);
                    if (f) { rflags = f; restart = true; break; }
                }
                if (tid == 0) S.ncand = 0;
                // (b) claim never-seen diagonals; every predecessor of this
                // round folds its (W, t) into the slot with a max
                for (int32_t base = 0; base < nc; base += BLOCK) {
                    const int32_t c = base + tid;
                    int claim = 0;
                    if (c < nc) {
                        const int ds = cd[c];
                        Page* pg = &pages[ds];
                        const int sl = ck[c] & 31;
                        const int32_t st = __hip_atomic_load(&pg->stamp[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        bool part = false;
                        if (st == ST_EMPTY) {
                            const int32_t old = atomicCAS(&pg->stamp[sl], ST_EMPTY, ST_CLAIM);
                            if (old == ST_EMPTY) { claim = 1; part = true; }
                            else if (old == ST_CLAIM) part = true;
                        } else if (st == ST_CLAIM) {
                            part = true;
                        }
                        if (part) atomicMax(&pg->wt[sl], pack_wt(cW[c], ct[c]));
                    }
                    const int pos = wave_alloc(claim, &S.n[b]);
                    if (claim) {
                        if (pos < A.list_cap) {
                            L[b].v[pos] = cu[c]; L[b].k[pos] = ck[c]; L[b].o[pos] = 0;
                            L[b].w[pos] = 0; L[b].t[pos] = -1; L[b].d[pos] = cd[c];
                        } else {
                            atomicOr(&S.flags, F_LIST);
                        }
                    }
                }
                __syncthreads();
                const int32_t hi_next = S.n[b];
                {
                    const int f = read_uniform(S.flags);
                    if (f) { rflags = f; restart = true; break; }
                }
                lo = hi;
                hi = hi_next;
                if (tid == 0) S.cross += (ull)(hi - lo);
            }
            if (restart) break;
            if (chunks) atomicAdd(&S.chunks, (ull)chunks);
            const int32_t n = S.n[b];
            work += n;
            // ================= END TEST =================
            if (S.found) { status = GWFA_ST_OK; break; }
            if (A.max_score >= 0 && s >= A.max_score) { status = GWFA_ST_MAX_SCORE; break; }
            // cannot happen for valid input (the query can always be
            // inserted); a guard so that every workgroup finishes
            if (n == 0 || s > qlen + 1) { status = GWFA_ST_MAX_SCORE; break; }
            int32_t ncur = n;
            // ================= PRUNE (Algorithm 4) =================
            if (A.prune == GWFA_PRUNE_HEURISTIC && S.amax > A.a_diff) {
                const int nb = 1 - b;
                const int32_t amax = S.amax;
                __syncthreads();
                if (tid == 0) S.n[nb] = 0;
                __syncthreads();
                for (int32_t base = 0; base < ncur; base += BLOCK) {
                    const int32_t idx = base + tid;
                    int keep = 0;
                    if (idx < ncur) {
                        const int32_t a = L[b].k[idx] + L[b].o[idx] + L[b].w[idx];
                        keep = (amax - a < A.a_diff) ? 1 : 0;
                        if (!keep) {
                            const int32_t ds = L[b].d[idx], k = L[b].k[idx];
                            pages[ds].stamp[k & 31] = s | ST_PRUNED;   // record kept, not in F_s
                        }
                    }
                    const int pos = wave_alloc(keep, &S.n[nb]);
                    if (keep) {
                        L[nb].v[pos] = L[b].v[idx]; L[nb].k[pos] = L[b].k[idx]; L[nb].o[pos] = L[b].o[idx];
                        L[nb].w[pos] = L[b].w[idx]; L[nb].t[pos] = L[b].t[idx]; L[nb].d[pos] = L[b].d[idx];
                    }
                }
                __syncthreads();
                if (tid == 0) S.dropped += ncur - S.n[nb];
                b = nb;
                ncur = S.n[b];
            }
            // ================= EXPAND (Algorithm 3) =================
            {
                const int nb = 1 - b;
                __syncthreads();
                if (tid == 0) S.n[nb] = 0;
                __syncthreads();
                int adm = 0;
                for (int32_t base = 0; base < ncur; base += BLOCK) {
                    const int32_t idx = base + tid;
                    int cnt = 0;
                    int32_t ok[3], oo[3], ow[3], ot[3], od[3];
                    int32_t v = 0;
                    if (idx < ncur) {
                        v = L[b].v[idx];
                        const int32_t k = L[b].k[idx], o0 = L[b].o[idx], W0 = L[b].w[idx], t0 = L[b].t[idx];
                        const int32_t ds0 = L[b].d[idx];
                        const int32_t Lv = (int32_t)(seg_off[v + 1] - seg_off[v]);
                        const int32_t i0 = k + o0;
                        const int sl = k & 31;
                        const int32_t kp0 = k >> 5;
                        const int pl = (sl < 2) ? dir_find(dir, mask, dkey(v, kp0 - 1)) : -1;
                        const int ph = (sl > 29) ? dir_find(dir, mask, dkey(v, kp0 + 1)) : -1;
                        // neighbours d = -2, -1, +1, +2 -> j = 0, 1, 2, 3
                        int32_t nst[4], nof[4], npg[4];
                        ull nwt[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int d = (j < 2) ? (j - 2) : (j - 1);
                            const int x = sl + d;
                            const int p = (x < 0) ? pl : ((x > 31) ? ph : ds0);
                            npg[j] = p;
                            if (p >= 0) {
                                const int xs = x & 31;
                                nst[j] = pages[p].stamp[xs];
                                nof[j] = pages[p].off[xs];
                                nwt[j] = (j >= 2 && nst[j] == s) ? pages[p].wt[xs] : 0ull;
                            } else {
                                nst[j] = ST_EMPTY; nof[j] = 0; nwt[j] = 0ull;
                            }
                        }
                        const bool pm2 = nst[0] == s, pm1 = nst[1] == s, pp1 = nst[2] == s, pp2 = nst[3] == s;
                        // output k+1: insertion from k, mismatch at k+1, deletion from k+2
                        {
                            int32_t bo = -1, bw = -1, bt = -1;
                            if (i0 < qlen) { bo = o0; bw = W0; bt = t0; }
                            if (pp1) {
                                const int32_t o1 = nof[2];
                                if (k + 1 + o1 < qlen && o1 < Lv) {
                                    const int32_t w1 = wt_W(nwt[2]) + 1;
                                    if (o1 + 1 > bo || (o1 + 1 == bo && w1 > bw)) { bo = o1 + 1; bw = w1; bt = wt_t(nwt[2]); }
                                }
                            }
                            if (pp2) {
                                const int32_t o2 = nof[3];
                                if (o2 < Lv) {
                                    const int32_t w2 = wt_W(nwt[3]) + 1;
                                    if (o2 + 1 > bo || (o2 + 1 == bo && w2 > bw)) { bo = o2 + 1; bw = w2; bt = wt_t(nwt[3]); }
                                }
                            }
                            const bool rec = nst[2] != ST_EMPTY;
                            if (bo >= 0 && (!rec || bo > nof[2])) {
                                ok[cnt] = k + 1; oo[cnt] = bo; ow[cnt] = bw; ot[cnt] = bt; od[cnt] = npg[2]; ++cnt;
                            }
                        }
                        // output k (owned when k-1 is absent): mismatch at k, deletion from k+1
                        if (!pm1) {
                            int32_t bo = -1, bw = -1, bt = -1;
                            if (i0 < qlen && o0 < Lv) { bo = o0 + 1; bw = W0 + 1; bt = t0; }
                            if (pp1 && nof[2] < Lv) {
                                const int32_t o1 = nof[2] + 1, w1 = wt_W(nwt[2]) + 1;
                                if (o1 > bo || (o1 == bo && w1 > bw)) { bo = o1; bw = w1; bt = wt_t(nwt[2]); }
                            }
                            if (bo > o0) { ok[cnt] = k; oo[cnt] = bo; ow[cnt] = bw; ot[cnt] = bt; od[cnt] = ds0; ++cnt; }
                        }
                        // output k-1 (owned when k-1 and k-2 are absent): deletion from k
                        if (!pm1 && !pm2 && o0 < Lv) {
                            const bool rec = nst[1] != ST_EMPTY;
                            if (!rec || o0 + 1 > nof[1]) {
                                ok[cnt] = k - 1; oo[cnt] = o0 + 1; ow[cnt] = W0 + 1; ot[cnt] = t0; od[cnt] = npg[1]; ++cnt;
                            }
                        }
                    }
                    const int pos = wave_alloc(cnt, &S.n[nb]);
                    for (int j = 0; j < cnt; ++j) {
                        const int32_t p = pos + j;
                        if (p < A.list_cap) {
                            L[nb].v[p] = v; L[nb].k[p] = ok[j]; L[nb].o[p] = oo[j];
                            L[nb].w[p] = ow[j]; L[nb].t[p] = ot[j]; L[nb].d[p] = od[j];
                        } else {
                            atomicOr(&S.flags, F_LIST);
                        }
                    }
                    adm += cnt;
                }
                if (adm) atomicAdd(&S.adm, (ull)adm);
                {
                    const int f = read_uniform(S.flags);
                    if (f) { rflags = f; restart = true; break; }
                }
                const int32_t nn = S.n[nb];
                // pages for admitted diagonals that have none yet
                for (int32_t idx = tid; idx < nn; idx += BLOCK) {
                    if (L[nb].d[idx] < 0) {
                        bool ins;
                        const int ds = dir_insert(dir, mask, dkey(L[nb].v[idx], L[nb].k[idx] >> 5), ins);
                        if (ds < 0) atomicOr(&S.flags, F_GROW);
                        else if (ins) { page_init(&pages[ds]); atomicAdd(&S.dirn, 1); }
                        L[nb].d[idx] = ds;
                    }
                }
                __syncthreads();
                rflags = S.flags | ((S.dirn > (int32_t)((mask + 1) >> 1)) ? F_GROW : 0);
                if (rflags) { restart = true; break; }
                b = nb;
            }
        }
        if (!restart) break;
        // capacity exceeded: grow the directory if possible, else give up
        const int fl = rflags;
        __syncthreads();
        if ((fl & F_GROW) && !(fl & F_LIST) && cap_log2 + 2 <= A.dir_log2_max) {
            cap_log2 += 2;
            continue;
        }
        if ((fl & F_GROW) && !(fl & F_LIST) && cap_log2 < A.dir_log2_max) {
            cap_log2 = A.dir_log2_max;
            continue;
        }
        status = GWFA_ST_ARENA;
        break;
    }
    // ================= results and walk (Algorithm 6) =================
    if (status == GWFA_ST_OK && tb) {
        if (tid == 0) S.tend = -1;
        __syncthreads();
        const int32_t ev = (int32_t)(S.endkey >> 32), eo = (int32_t)(S.endkey & 0xffffffffull);
        const int32_t n = S.n[b];
        for (int32_t idx = tid; idx < n; idx += BLOCK)
            if (L[b].v[idx] == ev && L[b].o[idx] == eo && L[b].k[idx] + eo == qlen) S.tend = L[b].t[idx];
        __syncthreads();
    }
    if (tid == 0) {
        out->status = status;
        out->n_scores = s + 1;
        out->work = work;
        out->path_off = -1;
        out->path_len = 0;
        if (status == GWFA_ST_OK) {
            out->dist = s;
            out->end_v = (int32_t)(S.endkey >> 32);
            out->end_off = (int32_t)(S.endkey & 0xffffffffull);
            if (tb && S.tend >= 0) {
                int32_t len = 0;
                for (int32_t t = S.tend; t >= 0; t = Tt[t]) ++len;
                const ull pos = atomicAdd(A.path_cursor, (ull)len);
                out->path_len = len;
                if ((int64_t)pos + len <= A.path_cap && A.path_buf) {
                    int32_t j = len - 1;
                    for (int32_t t = S.tend; t >= 0; t = Tt[t]) A.path_buf[pos + (j--)] = Tv[t];
                    out->path_off = (int64_t)pos;
                }
            }
        } else {
            out->dist = -1; out->end_v = -1; out->end_off = -1;
            if (status == GWFA_ST_ARENA && A.retry) {
                const int ri = atomicAdd(A.retry_count, 1);
                A.retry[ri] = r;
            }
        }
        if (A.stats) {
            atomicAdd(&A.stats[0], (ull)work);
            atomicAdd(&A.stats[1], S.cross);
            atomicAdd(&A.stats[2], (ull)S.dirn);
            atomicAdd(&A.stats[3], S.chunks);
            atomicAdd(&A.stats[4], S.adm);
            atomicAdd(&A.stats[6], S.mlp);
            atomicAdd(&A.stats[7], (ull)S.dropped);
        }
    }
    __syncthreads();
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_align(KArgs A) {
    __shared__ Shared S;
    char* arena = A.arena + (int64_t)blockIdx.x * A.arena_stride;
    for (;;) {
        if (threadIdx.x == 0) S.read = atomicAdd(A.queue, 1);
        __syncthreads();
        const int ridx = S.read;
        __syncthreads();
        if (ridx >= A.n_reads) break;
        const int r = A.order ? A.order[ridx] : ridx;
        align_read<BLOCK>(A, arena, r, S);
    }
}

// ASCII -> 2-bit packed words; one thread per output word (32 bases).
__global__ void k_pack(const uint8_t* __restrict__ ascii, int64_t n, ull* __restrict__ out, int64_t n_words,
                       int32_t* err) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_words) return;
    const int64_t b0 = w * 32;
    ull word = 0;
    int bad = 0;
    if (b0 + 32 <= n && ((reinterpret_cast<uintptr_t>(ascii + b0) & 15) == 0)) {
        const uint4* p = reinterpret_cast<const uint4*>(ascii + b0);
        const uint4 x0 = p[0], x1 = p[1];
        const uint32_t wd[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t ch = (wd[j] >> (8 * c)) & 0xffu;
                const uint32_t u = ch & 0xdfu;   // upper case
                const uint32_t code = (u == 'A') ? 0u : (u == 'C') ? 1u : (u == 'G') ? 2u : (u == 'T') ? 3u : 4u;
                bad |= code == 4u;
                word = (word << 2) | (ull)(code & 3u);
            }
        }
    } else {
        for (int j = 0; j < 32; ++j) {
            const int64_t bi = b0 + j;
            uint32_t code = 0;
            if (bi < n) {
                const uint32_t u = ascii[bi] & 0xdfu;
                code = (u == 'A') ? 0u : (u == 'C') ? 1u : (u == 'G') ? 2u : (u == 'T') ? 3u : 4u;
                bad |= code == 4u;
            }
            word = (word << 2) | (ull)(code & 3u);
        }
    }
    out[w] = word;
    if (bad && err) atomicExch(err, (int32_t)GWFA_ERR_ALPHABET);
}

__global__ void k_reset(int32_t* queue, ull* path_cursor, int32_t* retry_count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *queue = 0;
        if (path_cursor) *path_cursor = 0;
        if (retry_count) *retry_count = 0;
    }
}

}  // namespace gwfa_dev

// ---------------------------------------------------------------------------
// launch helpers (called from the host code)
// ---------------------------------------------------------------------------
hipError_t gwfa_launch_align(const KArgs& A, int lanes, int groups, hipStream_t st) {
    switch (lanes) {
    case 64: hipLaunchKernelGGL(gwfa_dev::k_align<64>, dim3(groups), dim3(64), 0, st, A); break;
    case 128: hipLaunchKernelGGL(gwfa_dev::k_align<128>, dim3(groups), dim3(128), 0, st, A); break;
    case 256: hipLaunchKernelGGL(gwfa_dev::k_align<256>, dim3(groups), dim3(256), 0, st, A); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t gwfa_launch_pack(const uint8_t* ascii, int64_t n, unsigned long long* out, int64_t n_words, int32_t* err,
                            hipStream_t st) {
    if (n_words <= 0) return hipSuccess;
    const int tpb = 256;
    const int64_t blocks = (n_words + tpb - 1) / tpb;
    hipLaunchKernelGGL(gwfa_dev::k_pack, dim3((unsigned)blocks), dim3(tpb), 0, st, ascii, n, out, n_words, err);
    return hipGetLastError();
}

hipError_t gwfa_launch_reset(int32_t* queue, unsigned long long* cursor, int32_t* retry_count, hipStream_t st) {
    hipLaunchKernelGGL(gwfa_dev::k_reset, dim3(1), dim3(64), 0, st, queue, cursor, retry_count);
    return hipGetLastError();
}
