// gwfa_kernels.hip -- device code of the graph wavefront alignment library
// for AMD CDNA4 (gfx950).
//
// One persistent workgroup aligns one query at a time, taking queries from a
// device work queue.  Per score s it runs the paper's loop (Section 2.4):
//   EXPAND  (Algorithm 3): insertion / deletion / mismatch candidates of every
//           diagonal of F_s, merged per diagonal, admitted when they beat the
//           diagonal's record;
//   EXTEND  (Algorithm 2): every admitted diagonal slides along its vertex by
//           the exact-match run (2-bit packed XOR + count-leading-zeros, 32
//           bases per step); a diagonal reaching the end of vertex v creates
//           (u, k+|v|) at offset 0 on every out-edge (v,u) not seen before, at
//           the same score (cost 0), and those are extended in further rounds;
//   END     (extension mode): stop at the first score at which a wavefront
//           cell has consumed the whole query;
//   PRUNE   (Algorithm 4, optional) or the learned keep/drop network.
//
// The wavefront F_s is a list sorted by (v, k).  The expansion is
// owner-computes: output diagonal k' of vertex v is produced by the present
// source with the smallest k among k'-1, k', k'+1, and those sources are the
// source's neighbours in the sorted list, so the expansion reads no table
// except at the two ends of a run of consecutive diagonals (where the record
// of a diagonal outside F_s decides).  Outputs come out sorted (ordered block
// scan) and are extended by the lane that produced them in the same pass.
// Diagonals created by crossings are sorted (bitonic) and merged in.
//
// Records of the paper's wavefront set H~ (kept for the life of a query):
// pages of 32 consecutive diagonals of one vertex, found through an
// open-addressing directory keyed (v, k >> 5).  A record word is
// (generation << 32 | offset): a word whose generation is not the current
// query's is "never seen", so pages need no initialisation.  A record holds
// the diagonal's offset when it left the wavefront (reached the vertex end,
// consumed the query, or was pruned) -- the only diagonals outside F_s that
// can still be candidates.
//
// Global form (an end vertex v_e): the end test is Algorithm 1's, the cell
// (|q|, v_e, |v_e|); diagonals that consumed the query go on by deletions
// and crossings; an empty wavefront means v_e cannot be reached.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "gwfa_internal.h"
#include "gwfa_mlp_dev.h"

namespace gwfa_dev {

using namespace gwfa_nn;

typedef unsigned long long ull;

constexpr int PAGE = 32;
constexpr int32_t CLAIM_BASE = 0x40000000;   // record value while a crossing round claims it
constexpr int F_GROW = 1;   // directory / trace capacity exceeded: restart with a bigger one
constexpr int F_LIST = 2;   // list / candidate capacity exceeded: re-run on a larger tier
// Crossing entries sorted in LDS (virtual merge) up to this many per
// workgroup of `block` lanes; larger sets are sorted in the arena.
constexpr int xs_lds(int block) { return block >= 256 ? 1024 : 4 * block; }
// The expansion writes the sort key of every SAMP-th entry of the list it
// builds into LDS (up to NSAMP keys): the merge then finds an entry's place
// in that list by a search in LDS and one round of at most SAMP-1 loads.
constexpr int SAMP = 8;
constexpr int nsamp(int block) { return block >= 256 ? 1024 : 256; }
// The exact mode stages the crossing rounds' data in LDS: up to xstage(block)
// diagonals claimed by one round (read back by the next round's extension)
// and up to twice as many crossing candidates (read back by the claims); the
// rest goes through the arena.
constexpr int xstage(int block) { return block >= 512 ? 256 : (block >= 256 ? 128 : 64); }


struct Page {
    ull R[PAGE];    // (gen << 32) | record offset (or CLAIM_BASE + round)
    ull Wc[PAGE];   // (gen << 32) | W: max walk length of a round's crossings
};
static_assert(sizeof(Page) == 512, "page layout");

__device__ __forceinline__ ull mkR(uint32_t gen, int32_t r) { return ((ull)gen << 32) | (ull)(uint32_t)r; }
__device__ __forceinline__ uint32_t rgen(ull w) { return (uint32_t)(w >> 32); }
__device__ __forceinline__ int32_t rval(ull w) { return (int32_t)(uint32_t)(w & 0xffffffffull); }

__device__ __forceinline__ ull dkey(int32_t v, int32_t kp) {
    return ((ull)(uint32_t)(v + 1) << 32) | (ull)(uint32_t)(kp + 0x40000000);
}
__device__ __forceinline__ ull skey(int32_t v, int32_t k) {   // sort key of a diagonal
    return ((ull)(uint32_t)v << 32) | (ull)(uint32_t)(k + 0x40000000);
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

// LCP of q[qp ...] and label[sp ...], at most lim bases.  Each step
// compares up to four consecutive 32-base windows; they share words (window j
// spans words j and j+1 of the step), so a step loads five words per
// sequence, all issued together: a long exact run costs one memory round trip
// per 128 bases.  Word indices are clamped to qmax / smax, the word after the
// one holding the range's last base (both stores end with two words of
// padding, so that word exists): a window that starts inside the range never
// reaches past it, and the words clamped are never used.
// ALL = false loads only the words the step needs (fewer registers in
// flight, for call sites where registers are scarce).
template <bool ALL = true>
__device__ __forceinline__ int32_t lcp(const ull* __restrict__ qw, int64_t qp, int64_t qmax, const ull* __restrict__ sw,
                                       int64_t sp, int64_t smax, int32_t lim, uint32_t& chunks) {
    int32_t l = 0;
    const int qs = (int)((qp & 31) * 2), ss = (int)((sp & 31) * 2);
    while (l < lim) {
        const int32_t rem = lim - l;
        const int64_t qi = (qp + l) >> 5, si = (sp + l) >> 5;
        ull a[5], b[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            if (ALL) {
                a[j] = qw[min(qi + j, qmax)];
                b[j] = sw[min(si + j, smax)];
            } else {
                const bool need = 32 * (j - 1) < rem;   // word j is needed by windows j-1 and j
                a[j] = need ? qw[qi + j] : 0ull;
                b[j] = need ? sw[si + j] : 0ull;
            }
        }
        int32_t m = 0;
        bool stop = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!stop && 32 * j < rem) {
                ++chunks;
                const ull xq = (a[j] << qs) | ((a[j + 1] >> 1) >> (63 - qs));
                const ull xs = (b[j] << ss) | ((b[j + 1] >> 1) >> (63 - ss));
                const ull x = xq ^ xs;
                if (x) { m += (int32_t)(__clzll((long long)x) >> 1); stop = true; }
                else m += 32;
            }
        }
        if (m >= rem) return lim;
        l += m;
        if (stop) return l;
    }
    return l;
}

__device__ int dir_find(const ull* __restrict__ dir, uint32_t mask, ull key) {
    uint32_t h = dhash(key) & mask;
    for (uint32_t p = 0; p <= mask; ++p) {
        const ull c = __hip_atomic_load(&dir[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (c == key) return (int)h;
        if (c == 0) return -1;
        h = (h + 1) & mask;
    }
    return -1;
}

// Find-or-insert; counts insertions in *n_ins.  -1 when the table is full.
// The same, continuing from `c`, a value read from slot h earlier (it may be
// stale: a slot only ever goes from empty to a key, and an empty slot is
// claimed by compare-and-swap, which sees the current value).
__device__ int dir_settle(ull* dir, uint32_t mask, ull key, uint32_t h, ull c, int* n_ins) {
    for (uint32_t p = 0; p <= mask; ++p) {
        if (p > 0) c = __hip_atomic_load(&dir[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (c == key) return (int)h;
        if (c == 0) {
            const ull old = atomicCAS(&dir[h], 0ull, key);
            if (old == 0) { atomicAdd(n_ins, 1); return (int)h; }
            if (old == key) return (int)h;
        }
        h = (h + 1) & mask;
    }
    return -1;
}
__device__ __forceinline__ int dir_insert(ull* dir, uint32_t mask, ull key, int* n_ins) {
    const uint32_t h = dhash(key) & mask;
    return dir_settle(dir, mask, key, h, __hip_atomic_load(&dir[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), n_ins);
}

// Exclusive prefix sum of x >= 0 over the 64 lanes of the wave, plus the
// total.  Bit plane b adds 2^b times the number of lower lanes that have
// bit b set (ballot + mbcnt): no data moves between lanes, one ballot per
// bit plane in use (the counts here are small: outputs, claims, keeps).
__device__ __forceinline__ int wave_excl_scan(int x, int& total) {
    uint32_t rem = (uint32_t)x;
    int ex = 0, tot = 0;
    for (int b = 0; __ballot(rem != 0u); ++b, rem >>= 1) {
        const ull m = __ballot(rem & 1u);
        ex += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) << b;
        tot += __popcll(m) << b;
    }
    total = tot;
    return ex;
}

// Reserves cnt consecutive slots of an LDS counter (one atomic per wave,
// order between waves unspecified).  All lanes of the wave must call it.
__device__ __forceinline__ int wave_alloc(int cnt, int* counter) {
    int total;
    const int ex = wave_excl_scan(cnt, total);
    int base = 0;
    if (__lane_id() == 0 && total > 0) base = atomicAdd(counter, total);
    // lane 0's value to every lane: a lane read (one ALU instruction), not a
    // permute through LDS
    base = __builtin_amdgcn_readlane(base, 0);
    return base + ex;
}

// Workgroup barrier for phases that exchange only LDS data: waits for this
// wave's LDS operations, not for its outstanding global stores (which the
// full __syncthreads() would drain).
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// A 64-bit value that is the same in every lane, as a scalar.
__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Exclusive prefix sum over the whole block in thread order (keeps lists
// sorted).  All threads must call it.
template <int BLOCK>
__device__ __forceinline__ int block_excl_scan(int x, int& total, int* scan) {
    constexpr int NW = BLOCK / 64;
    int wt;
    const int ex = wave_excl_scan(x, wt);
    const int w = threadIdx.x >> 6;
    if (NW == 1) { total = __builtin_amdgcn_readfirstlane(wt); return ex; }
    if (__lane_id() == 0) scan[w] = wt;
    lds_barrier();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const int y = scan[i];
        off += (i < w) ? y : 0;
        tot += y;
    }
    lds_barrier();
    total = __builtin_amdgcn_readfirstlane(tot);   // block-uniform: kept in a scalar register
    return off + ex;
}

// Reads a shared word that other threads may update in the phase that just
// ended, so that every thread takes the same decision: barrier, read,
// barrier (nobody can write it again before everybody has read it).
__device__ __forceinline__ int read_uniform(const int& x) {
    __syncthreads();
    const int v = *(const volatile int*)&x;
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(v);
}

// A wavefront list: per entry the diagonal (v, k), its offset o and record
// page d in one 16-byte word, the walk length W and the trace index t in
// arrays of their own (each moved only by the modes that use it).  The label
// length l and base b of v are kept only for the diagonals a crossing round
// creates (their extension in the next round then needs no lookup); every
// other reader takes them from the graph's per-vertex label record.
struct Lists {
    int4* e;          // (v, k, o, d)
    int32_t *w, *t, *l;
    int64_t* b;
};
// The diagonal (v, k) of entry i (the first 8 bytes of its word).
__device__ __forceinline__ int2 vk_of(const Lists& L, int32_t i) {
    return *reinterpret_cast<const int2*>(&L.e[i]);
}
// Label base of a per-vertex label record.
__device__ __forceinline__ int64_t lab_base(int4 lab) {
    return (int64_t)(((uint64_t)(uint32_t)lab.y << 32) | (uint32_t)lab.x);
}

// Workgroup LDS, sized for the workgroup (merge keys, the staged batch) and
// the mode (the network's weights only where it runs).
template <int BLOCK, int MODE>
struct Shared {
    static constexpr int XS = xs_lds(BLOCK);
    static constexpr int NB = BLOCK + 4;
    static constexpr int XC = MODE == 0 ? xstage(BLOCK) : 0;       // claimed diagonals staged
    static constexpr int CS = MODE == 0 ? 2 * xstage(BLOCK) : 0;   // crossing candidates staged
    int32_t read;
    int32_t n_out;    // entries in the list being built (outputs, then crossing entries)
    int32_t ncand;
    int32_t dirn;     // pages created
    int32_t mn;       // trace entries created
    int32_t flags;
    int32_t found;
    int32_t iend;     // largest end row reached (free end gap in the query)
    int32_t amax;
    int32_t imax;
    int32_t dropped;
    int32_t tend;
    uint32_t gen;
    ull endkey;
    ull chunks;
    ull cross;
    ull adm;
    ull mlp;
    ull tick[4];      // wall-clock ticks per phase (thread 0)
    int32_t scan[16];
    ull skeys[XS];
    int32_t sidx[XS];
    int32_t xcnt[XS];       // merge: main-list entries below each crossing entry
    ull samp[nsamp(BLOCK)]; // sort keys of list entries 0, SAMP, 2 SAMP, ... written by the expansion
    // expansion: the entries of one batch of the source list at slots 2 ..
    // BLOCK+1 plus two neighbours on each side (slots 0, 1, BLOCK+2, BLOCK+3)
    int32_t nbv[NB], nbk[NB], nbo[NB], nbd[NB], nbw[NB], nbt[NB];
    // crossing rounds: claimed diagonals (vertex, diagonal, page, label length,
    // predecessor's trace index, label base) and candidates (target, diagonal,
    // trace index of the crossing diagonal)
    int32_t xsv[XC + 1], xsk[XC + 1], xsd[XC + 1], xsl[XC + 1], xst[XC + 1];
    int64_t xsb[XC + 1];
    int32_t csu[CS + 1], csk[CS + 1], cst[CS + 1];
    alignas(16) uint16_t mlpw[MODE >= 2 ? 4808 : 8];   // pruning network (bfloat16), loaded once per launch
    float mscale[8];        // feature scales
};

// Per-query view of the arena and of the read.
struct Q {
    const ull* rd;
    int64_t q0;
    int32_t qlen, vs;
    int32_t j0, j1;   // start window: the walk starts after the first j bases of vs, j0 <= j <= j1
    int32_t ve;       // end vertex (global form) or -1 (extension mode)
    int32_t ilo;      // end rows: ilo .. qlen (qlen minus the free end gap in the query)
    bool wfree;       // global form: the walk may end anywhere inside ve
    ull* dir;
    Page* pages;
    ull* mkey;
    int32_t* Tv;
    int32_t* Tt;
    uint32_t mask;
    uint32_t gen;
    bool tb, track;   // traced walks; walk lengths and lags tracked (pruning, dumps)
};

template <class SH>
__device__ __forceinline__ int32_t trace_push_from(const Q& q, SH& S, int32_t v, int32_t tprev, ull probe);
// Algorithm 5: T gets (v, t) unless the pair is already there; the index of
// the pair's slot in the de-duplication map is its trace index.
template <class SH>
__device__ __forceinline__ int32_t trace_push(const Q& q, SH& S, int32_t v, int32_t tprev) {
    return trace_push_from(q, S, v, tprev,
                           __hip_atomic_load(&q.mkey[dhash(dkey(v, tprev)) & q.mask], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT));
}
// The same, given the value an earlier read found in the pair's first map
// slot (so that the read can go out with other loads).
template <class SH>
__device__ __forceinline__ int32_t trace_push_from(const Q& q, SH& S, int32_t v, int32_t tprev, ull probe) {
    const int ms = dir_settle(q.mkey, q.mask, dkey(v, tprev), dhash(dkey(v, tprev)) & q.mask, probe, &S.mn);
    if (ms < 0) { atomicOr(&S.flags, F_GROW); return -1; }
    // the slot's (v, tprev) is fixed by its key, so every inserter may write it
    q.Tv[ms] = v;
    q.Tt[ms] = tprev;
    return ms;
}

// Whether the front cell (v, o) of a diagonal can end a walk (the label of v
// has Lv bases): extension mode, any cell; global form, the last cell of ve,
// or any cell of ve when the walk's end gap is free.  A cell (v, 0) ends a
// walk only as the start cell (vs, 0).
__device__ __forceinline__ bool ends_walk(const Q& q, int32_t v, int32_t o, int32_t Lv) {
    if (q.ve >= 0 && (v != q.ve || (!q.wfree && o != Lv))) return false;
    return o >= 1 || (v == q.vs && q.j0 == 0);
}

// Records an extended diagonal: its record word when it is new or reached
// the vertex end, the end test and the pruning reductions; returns the number
// of out-edges to cross (0 unless the vertex end was reached).
template <class SH>
__device__ __forceinline__ int record_entry(const Q& q, SH& S, int32_t v, int32_t k, int32_t o, int32_t W,
                                            int32_t d, bool mark, int32_t Lv, int32_t deg, int2& lmax) {
    const int32_t i = k + o;
    // the record is written when the diagonal is new or may leave the
    // wavefront: at the vertex end, or with the query consumed (no mismatch
    // can advance it; in the global form the search goes on past i = |q|)
    if (mark || o == Lv || i == q.qlen) q.pages[d].R[k & 31] = mkR(q.gen, o);
    // end test: extension mode, any cell of the last query row; global form,
    // the cell at the end of the end vertex (Algorithm 1), or any cell of
    // the end vertex with a free end gap in the walk.  Offset-0 cells end a
    // walk only at the start cell (vs, 0): another one is the copy of a
    // predecessor's last cell.  With a free end gap in the query every row
    // from ilo on ends: the largest row reached is found here, its smallest
    // end cell once the score is complete.
    if (i >= q.ilo && ends_walk(q, v, o, Lv)) {
        S.found = 1;
        if (q.ilo < q.qlen) atomicMax(&S.iend, i);
        else atomicMin(&S.endkey, ((ull)(uint32_t)v << 32) | (uint32_t)o);
    }
    // Algorithm 4's a = i + W~ and the furthest row: this lane's maxima of the
    // score, reduced over the wave and the workgroup once the score is extended
    if (q.track) {
        lmax.x = max(lmax.x, i + W);
        lmax.y = max(lmax.y, i);
    }
    return (o == Lv) ? deg : 0;
}

// Extends one admitted diagonal (Algorithm 2) and records it.
template <class SH>
__device__ __forceinline__ int extend_entry(const KArgs& A, const Q& q, SH& S, int32_t v, int32_t k,
                                            int32_t& o, int32_t& W, int32_t d, bool mark, int64_t sb,
                                            int32_t Lv, int32_t deg, uint32_t& chunks, int2& lmax) {
    const int32_t i = k + o;
    const int32_t lim = min(q.qlen - i, Lv - o);
    const int32_t l = lcp(q.rd, q.q0 + i, ((q.q0 + q.qlen) >> 5) + 1, A.seg, sb + o, ((sb + Lv) >> 5) + 1, lim, chunks);
    o += l;
    W += l;
    return record_entry(q, S, v, k, o, W, d, mark, Lv, deg, lmax);
}

// Crossing candidate c: target u, diagonal k2 in u, walk length W, trace
// index t.  The first SH::CS (exact mode) go to LDS, the rest to the arena.
template <class SH>
__device__ __forceinline__ void put_cand(SH& S, const KArgs& A, int32_t* cu, int32_t* ck, int32_t* cW, int32_t* ct,
                                         int c, int32_t u, int32_t k2, int32_t W, int32_t t) {
    if (c < SH::CS) {
        S.csu[c] = u; S.csk[c] = k2; S.cst[c] = t;
    } else if (c < A.cand_cap) {
        cu[c] = u; ck[c] = k2; cW[c] = W; ct[c] = t;
    } else {
        atomicOr(&S.flags, F_LIST);
    }
}
// The candidates for the out-edges of a vertex whose out-edge record is vi
// (first edge, degree, first two targets), from slot c on.  Only the edges
// after the second need loads, in a branch of their own that ends by waiting
// for them: with a load inside the loop over all edges, or one possibly in
// flight after it, the compiler made the wave wait for every outstanding
// memory operation (the output stores and the next batch's entries among
// them) before each candidate, on every vertex.
template <class SH>
__device__ __forceinline__ void put_out_edges(SH& S, const KArgs& A, int32_t* cu, int32_t* ck, int32_t* cW,
                                              int32_t* ct, int c, int4 vi, int32_t k2, int32_t W, int32_t t) {
    const int deg = vi.y;
    if (deg > 0) put_cand(S, A, cu, ck, cW, ct, c, vi.z, k2, W, t);
    if (deg > 1) put_cand(S, A, cu, ck, cW, ct, c + 1, vi.w, k2, W, t);
    if (deg > 2) {
        for (int e = 2; e < deg; ++e) put_cand(S, A, cu, ck, cW, ct, c + e, A.out_dst[vi.x + e], k2, W, t);
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): no load of this branch outlives it
    }
}

// Bitonic sort of n keys (+ payload) in place, ascending; n is a power of 2.
// LDS=true when keys and payload are in LDS (stages then need LDS barriers only).
template <int BLOCK, bool LDS>
__device__ void bitonic(ull* keys, int32_t* idx, int n) {
    for (int kk = 2; kk <= n; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n; i += BLOCK) {
                const int p = i ^ j;
                if (p > i) {
                    const ull a = keys[i], b = keys[p];
                    const bool up = (i & kk) == 0;
                    if ((a > b) == up) {
                        keys[i] = b; keys[p] = a;
                        const int32_t t = idx[i]; idx[i] = idx[p]; idx[p] = t;
                    }
                }
            }
            if (LDS) lds_barrier(); else __syncthreads();
        }
    }
}

// Number of entries of list L[0, n) whose key is below key.
__device__ __forceinline__ int32_t lower_bound_list(const Lists& L, int32_t n, ull key) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        const int2 a = vk_of(L, mid);
        if (skey(a.x, a.y) < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}
// The same with the list's sampled keys in LDS (samp[j] = key of entry
// SAMP*j for j < ns): a search of the samples, then the at most SAMP-1
// entries between two samples, loaded together.  Beyond the sampled part of
// the list it falls back to the search in the list.
__device__ __forceinline__ int32_t lower_bound_sampled(const Lists& L, int32_t n, ull key, const ull* samp,
                                                       int32_t ns) {
    int32_t lo = 0, hi = ns;                 // samples below key
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (samp[mid] < key) lo = mid + 1; else hi = mid;
    }
    if (lo == 0) return 0;                   // entry 0 is not below key
    const int32_t a = SAMP * (lo - 1) + 1;   // entry a-1 is below key
    if (lo == ns && SAMP * ns < n) {         // past the sampled part
        int32_t l2 = a, h2 = n;
        while (l2 < h2) {
            const int32_t mid = (l2 + h2) >> 1;
            const int2 a = vk_of(L, mid);
            if (skey(a.x, a.y) < key) l2 = mid + 1; else h2 = mid;
        }
        return l2;
    }
    const int32_t b = min(SAMP * lo, n);     // entry b is not below key (or b = n)
    int32_t c = a;
    // every lane loads all SAMP-1 keys (indices clamped to the list), so that
    // the loads go out together
#pragma unroll
    for (int32_t j = 0; j < SAMP - 1; ++j) {
        const int32_t e = a + j;
        const int2 x = vk_of(L, min(e, n - 1));
        c += (e < b && skey(x.x, x.y) < key) ? 1 : 0;
    }
    return c;
}

// Merged view of a list whose first n1 entries are sorted and whose last m
// entries (crossing diagonals, unsorted in memory) have known merged
// positions: a bitmap over the merged positions (bit p of word p >> 5 set when
// position p holds a crossing entry), the number of bits set below each word,
// and the physical slots of the crossing entries in merged order.  The slot of
// merged position p takes two independent LDS reads and a count.
__device__ __forceinline__ int32_t vm_phys_bm(const uint32_t* bm, const int32_t* pre, const int32_t* xidx, int32_t p) {
    const uint32_t word = bm[p >> 5];
    const int b = p & 31;
    const int32_t c = pre[p >> 5] + __popc(word & ((1u << b) - 1u));
    return ((word >> b) & 1u) ? xidx[c] : p - c;
}

__device__ __forceinline__ int32_t lower_bound_keys(const ull* keys, int32_t n, ull key) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (keys[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Copies entry i of a to slot j of b; W moves only when a pruning mode reads
// it, t only when walks are traced.
__device__ __forceinline__ void copy_entry(const Lists& a, int32_t i, const Lists& b, int32_t j, bool w, bool t) {
    b.e[j] = a.e[i];
    if (w) b.w[j] = a.w[i];
    if (t) b.t[j] = a.t[i];
}

// ---------------------------------------------------------------------------
// Learned keep/drop of wavefront diagonals.
//
// Eight features of a diagonal whose front cell is (i, v, off) at score s,
// with walk length W (a = i + W as in Algorithm 4), the largest a and i of the
// wavefront, the label length |v| and out-degree of v:
//   0 log1p(a_max - a)      lag behind the furthest diagonal
//   1 log1p(s)              score
//   2 log1p(outdeg(v))
//   3 log1p(i_max - i)      distance from the query frontier
//   4 log1p(|v| - off)      bases left in the vertex
//   5 sign * log1p(|W - i|) walk/query drift (deletions minus insertions)
//   6 i / |q|               progress
//   7 log1p(|q| - i)        query left
// each multiplied by a per-feature scale and rounded to bfloat16 before the
// network (gwfa_mlp_dev.h) scores the diagonal.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void entry_features(float* f, int32_t s, int32_t i, int32_t W, int32_t off, int32_t Lv,
                                               int32_t deg, int32_t amax, int32_t imax, int32_t qlen) {
    f[0] = log1pf((float)(amax - (i + W)));
    f[1] = log1pf((float)s);
    f[2] = log1pf((float)deg);
    f[3] = log1pf((float)(imax - i));
    f[4] = log1pf((float)(Lv - off));
    const int32_t dr = W - i;
    f[5] = dr >= 0 ? log1pf((float)dr) : -log1pf((float)(-dr));
    f[6] = qlen > 0 ? (float)i / (float)qlen : 0.0f;
    f[7] = log1pf((float)(qlen - i));
}

// MODE 0: exact; 1: walk lengths tracked (Algorithm 4); 2: trace dump (and
// the learned keep/drop); 3: learned keep/drop without the dump.  Each mode
// is its own instantiation so that the registers of what it does not use
// are not allocated.
template <int BLOCK, int MODE>
__device__ void align_read(const KArgs& A, char* __restrict__ arena, int r, Shared<BLOCK, MODE>& S) {
    using SH = Shared<BLOCK, MODE>;
    constexpr bool LEARN = MODE >= 2;
    constexpr bool DUMP = MODE == 2;
    const int tid = threadIdx.x;
    Q q;
    q.rd = A.rd;
    // The query's parameters are the same in every lane: readfirstlane keeps
    // them in scalar registers (and the test below a branch of the whole wave).
    q.q0 = uniform64(A.rd_off[r]);
    q.qlen = __builtin_amdgcn_readfirstlane((int32_t)(A.rd_off[r + 1] - q.q0));
    q.vs = __builtin_amdgcn_readfirstlane(A.v_start[r]);
    q.ve = __builtin_amdgcn_readfirstlane(A.v_end ? A.v_end[r] : A.end_vertex);
    q.j0 = __builtin_amdgcn_readfirstlane(A.v_off ? A.v_off[r] : 0);
    q.j1 = __builtin_amdgcn_readfirstlane(A.v_off_hi ? A.v_off_hi[r] : q.j0);
    q.ilo = max(0, q.qlen - A.end_free);
    q.wfree = A.walk_free != 0;
    gwfa_result* out = A.res + r;
    const int64_t t_begin = (int64_t)wall_clock64();
    const int64_t* __restrict__ seg_off = A.seg_off;
    // Every query here passed the screen pass (k_screen): its start vertex,
    // start window and end vertex are in range.
    const int32_t* __restrict__ out_dst = A.out_dst;
    const int4* __restrict__ vinfo = A.vinfo;
    q.dir = reinterpret_cast<ull*>(arena + A.o_dir);
    q.pages = reinterpret_cast<Page*>(arena + A.o_pages);
    q.mkey = reinterpret_cast<ull*>(arena + A.o_mkey);
    q.Tv = reinterpret_cast<int32_t*>(arena + A.o_tv);
    q.Tt = reinterpret_cast<int32_t*>(arena + A.o_tt);
    q.tb = A.traceback != 0;
    q.track = MODE >= 1;   // the launch picks MODE >= 1 when pruning or dumping
    uint32_t* hdr = reinterpret_cast<uint32_t*>(arena + A.o_hdr);
    int32_t* const lbase = reinterpret_cast<int32_t*>(arena + A.o_lists);
    const int64_t lcap = A.list_cap;
    // list j (0 or 1): entry words, W, t, and the crossing diagonals' labels
    // (9 words per entry of list_cap entries)
    auto LL = [&](int j) -> Lists {
        int32_t* p = lbase + (int64_t)j * 9 * lcap;
        Lists x;
        x.e = reinterpret_cast<int4*>(p);
        x.w = p + 4 * lcap; x.t = p + 5 * lcap; x.l = p + 6 * lcap;
        x.b = reinterpret_cast<int64_t*>(p + 7 * lcap);
        return x;
    };
    int32_t* cbase = reinterpret_cast<int32_t*>(arena + A.o_cand);
    const int64_t cc = A.cand_cap;
    int32_t *cu = cbase, *ck = cbase + cc, *cW = cbase + 2 * cc, *ct = cbase + 3 * cc;
    ull* gkeys = reinterpret_cast<ull*>(arena + A.o_sort);
    int32_t* gidx = reinterpret_cast<int32_t*>(gkeys + A.sort_cap);

    int cap_log2 = 8;
    {
        const int64_t want = ((int64_t)q.qlen / 32 + 1) * A.dir_factor;
        while (cap_log2 < A.dir_log2_max && ((int64_t)1 << cap_log2) < want) ++cap_log2;
    }
    int status = -1;
    int32_t s = 0;
    int32_t clip = 0;         // query bases left unaligned (free end gap)
    int cur = 1;
    int32_t n_cur = 0;
    int32_t vmx = 0;          // crossing entries of the source list merged virtually
    uint32_t* const vm_bits = reinterpret_cast<uint32_t*>(S.skeys);
    int32_t* const vm_pre = reinterpret_cast<int32_t*>(S.skeys) + SH::XS;
    int64_t work = 0;
    uint32_t chunks = 0;
    for (;;) {   // attempts with a growing directory
        const uint32_t mask = (1u << cap_log2) - 1;
        const int32_t half = (int32_t)((mask + 1) >> 1);
        q.mask = mask;
        for (uint32_t i = tid; i <= mask; i += BLOCK) {
            q.dir[i] = 0;
            if (q.tb) q.mkey[i] = 0;
        }
        if (tid == 0) {
            const uint32_t g = hdr[0] + 1;
            hdr[0] = g;
            S.gen = g;
            S.n_out = 0; S.ncand = 0; S.dirn = 0; S.mn = 0; S.flags = 0;
            S.chunks = 0; S.cross = 0; S.adm = 0; S.mlp = 0; S.dropped = 0;
            S.found = 0; S.iend = -1; S.endkey = ~0ull; S.amax = 0; S.imax = 0;
            S.tick[0] = S.tick[1] = S.tick[2] = S.tick[3] = 0;
        }
        __syncthreads();
        q.gen = __builtin_amdgcn_readfirstlane(S.gen);
        // score 0 starts from the start cells (0, vs, j), j0 <= j <= j1: diagonal
        // -j at offset j, sorted by k (t = 0 is j1).  A start's trace record is
        // (vs, -1 - j), so the traced walk tells where it started.
        {
            const int32_t nst = q.j1 - q.j0 + 1;
            const Lists L0 = LL(0);
            const int64_t sb0 = seg_off[q.vs];
            const int32_t lv0 = (int32_t)(seg_off[q.vs + 1] - sb0);
            for (int32_t t = tid; t < min(nst, (int32_t)A.list_cap); t += BLOCK) {
                const int32_t j = q.j1 - t;
                const int ds = dir_insert(q.dir, mask, dkey(q.vs, (-j) >> 5), &S.dirn);
                if (ds < 0) atomicOr(&S.flags, F_GROW);
                const int32_t t0 = q.tb ? trace_push(q, S, q.vs, -1 - j) : -1;
                L0.e[t] = make_int4(q.vs, -j, j, ds);
                L0.w[t] = 0; L0.t[t] = t0;
                L0.b[t] = sb0; L0.l[t] = lv0;
            }
            if (tid == 0) {
                S.n_out = min(nst, (int32_t)A.list_cap);
                if (nst > A.list_cap) atomicOr(&S.flags, F_LIST);
            }
        }
        __syncthreads();
        // a start window that does not fit restarts with more working memory
        const int f0 = __builtin_amdgcn_readfirstlane(S.flags | ((S.dirn > half || S.mn > half) ? F_GROW : 0));
        const int32_t n_start = __builtin_amdgcn_readfirstlane(S.n_out);
        __syncthreads();
        cur = 1;
        n_cur = 0;
        vmx = 0;
        s = 0;
        work = 0;
        status = -1;
        int rflags = f0;
        chunks = 0;
        for (;; ++s) {
            if (f0) break;
            const int nb = 1 - cur;
            const Lists Ld = LL(nb);
            int32_t n1 = 0;           // diagonals produced by the expansion
            int2 lmax = make_int2(0, 0);   // this lane's largest a = i + W~ and i of the score (tracked modes)
            ull tk = wall_clock64();
            if (s > 0) {
                if (tid == 0) { S.found = 0; S.iend = -1; S.endkey = ~0ull; S.amax = 0; S.imax = 0; }
                __syncthreads();
                // ========== EXPAND (Algorithm 3) + EXTEND of what it admits ==========
                const Lists Ls = LL(cur);
                const int32_t n = n_cur;
                int32_t outbase = 0;
                int adm = 0;
                // each batch's entries (and, in threads 0-3, the two neighbours on
                // each side of it) are loaded one batch ahead, before the stores
                // of the batch being processed, so that their arrival does not
                // wait for those stores
                int4 pe, ph;
                int32_t pw, pt, phw, pht;
                auto fetch_batch = [&](int32_t bb) {
                    pe = make_int4(-1, 0, 0, 0); pw = 0; pt = -1;
                    const int32_t ix = bb + tid;
                    if (ix < n) {
                        const int32_t p0 = vmx ? vm_phys_bm(vm_bits, vm_pre, S.sidx, ix) : ix;
                        pe = Ls.e[p0];
                        if (q.track) pw = Ls.w[p0];
                        if (q.tb) pt = Ls.t[p0];
                    }
                    ph = make_int4(-1, 0, 0, 0); phw = 0; pht = -1;
                    if (tid < 4) {
                        const int32_t hp = tid < 2 ? bb - 2 + tid : bb + BLOCK + (tid - 2);
                        if (hp >= 0 && hp < n) {
                            const int32_t pp = vmx ? vm_phys_bm(vm_bits, vm_pre, S.sidx, hp) : hp;
                            ph = Ls.e[pp];
                            if (q.track) phw = Ls.w[pp];
                            if (q.tb) pht = Ls.t[pp];
                        }
                    }
                };
                fetch_batch(0);
                for (int32_t base = 0; base < n; base += BLOCK) {
                    const int32_t idx = base + tid;
                    const bool valid = idx < n;
                    // three fixed output slots: diagonals k-1, k, k+1
                    bool ov0 = false, ov1 = false, ov2 = false;
                    int32_t oo0 = 0, ow0 = 0, ot0 = 0, od0 = -1; bool on0 = false;
                    int32_t oo1 = 0, ow1 = 0, ot1 = 0, od1 = -1;
                    int32_t oo2 = 0, ow2 = 0, ot2 = 0, od2 = -1; bool on2 = false;
                    // this lane's entry (merged position idx); v = -1 past the end
                    const int32_t v = pe.x, k = pe.y, o0 = pe.z, ds0 = pe.w, W0 = pw, t0 = pt;
                    // the label of v (its length bounds the candidates, its base places
                    // their windows), requested before the exchange of neighbours,
                    // which hides its latency
                    const int4 lab = A.vlab[valid ? v : 0];   // unconditional: its wait can move to the first use
                    // the neighbours at merged positions idx-2 .. idx+2 come from LDS:
                    // every lane stages its entry, threads 0-3 the two positions on
                    // each side of the batch
                    {
                        const int32_t hv = ph.x, hk = ph.y, ho = ph.z, hd = ph.w, hw = phw, ht = pht;
                        const int hs = tid < 2 ? tid : BLOCK + tid;
                        S.nbv[tid + 2] = v; S.nbk[tid + 2] = k; S.nbo[tid + 2] = o0; S.nbd[tid + 2] = ds0;
                        if (q.track) S.nbw[tid + 2] = W0;
                        if (q.tb) S.nbt[tid + 2] = t0;
                        if (tid < 4) {
                            S.nbv[hs] = hv; S.nbk[hs] = hk; S.nbo[hs] = ho; S.nbd[hs] = hd;
                            if (q.track) S.nbw[hs] = hw;
                            if (q.tb) S.nbt[hs] = ht;
                        }
                    }
                    lds_barrier();
                    const int32_t Lv = lab.z;
                    const int64_t sb = lab_base(lab);
                    const int32_t vm1 = S.nbv[tid + 1], km1 = S.nbk[tid + 1];
                    const int32_t vm2 = S.nbv[tid], km2 = S.nbk[tid];
                    const int32_t vp1 = S.nbv[tid + 3], kp1 = S.nbk[tid + 3], op1 = S.nbo[tid + 3];
                    const int32_t dp1 = S.nbd[tid + 3];
                    const int32_t vp2 = S.nbv[tid + 4], kp2 = S.nbk[tid + 4], op2 = S.nbo[tid + 4];
                    const int32_t wp1 = q.track ? S.nbw[tid + 3] : 0, wp2 = q.track ? S.nbw[tid + 4] : 0;
                    const int32_t tp1 = q.tb ? S.nbt[tid + 3] : -1, tp2 = q.tb ? S.nbt[tid + 4] : -1;
                    // candidate outputs (before the record checks) and their first
                    // 32-base windows, fetched together with the records
                    int32_t c0 = -1, c1 = -1, c2 = -1;    // candidate offsets, -1 = none
                    int32_t cw1 = -1, ct1 = -1, cw2 = -1, ct2 = -1;
                    bool rec0 = false, rec2 = false;      // needs a record check
                    int32_t d2 = -1;
                    int pg0 = -1, pg2 = -1;
                    if (valid) {
                        const int32_t i0 = k + o0;
                        // k-2, k-1 (k+1, k+2) of the same vertex are adjacent in the sorted list
                        const bool pm1 = vm1 == v && km1 == k - 1;
                        const bool pm2 = pm1 ? (vm2 == v && km2 == k - 2) : (vm1 == v && km1 == k - 2);
                        const bool pp1 = vp1 == v && kp1 == k + 1;
                        bool pp2;
                        int32_t o1 = 0, W1 = 0, t1 = 0, o2 = 0, W2 = 0, t2 = 0;
                        if (pp1) {
                            o1 = op1; W1 = wp1; t1 = tp1; d2 = dp1;
                            pp2 = vp2 == v && kp2 == k + 2;
                            o2 = op2; W2 = wp2; t2 = tp2;
                        } else {
                            pp2 = vp1 == v && kp1 == k + 2;
                            o2 = op1; W2 = wp1; t2 = tp1;
                        }
                        const int sl = k & 31;
                        const int32_t kp0 = k >> 5;
                        // output k-1 (this source owns it when k-1 and k-2 are absent): deletion
                        if (!pm1 && !pm2 && o0 < Lv) {
                            c0 = o0 + 1;
                            rec0 = true;
                            // a missing page means no record: the output is admitted and
                            // needs the page, so it is created now
                            pg0 = (sl > 0) ? ds0 : dir_insert(q.dir, mask, dkey(v, kp0 - 1), &S.dirn);
                        }
                        // output k (owned when k-1 is absent): mismatch, deletion from k+1
                        if (!pm1) {
                            int32_t bo = -1, bw = -1, bt = -1;
                            if (i0 < q.qlen && o0 < Lv) { bo = o0 + 1; bw = W0 + 1; bt = t0; }
                            if (pp1 && o1 < Lv && (o1 + 1 > bo || (o1 + 1 == bo && W1 + 1 > bw))) {
                                bo = o1 + 1; bw = W1 + 1; bt = t1;
                            }
                            if (bo > o0) { c1 = bo; cw1 = bw; ct1 = bt; }
                        }
                        // output k+1 (always owned): insertion, mismatch at k+1, deletion from k+2
                        {
                            int32_t bo = -1, bw = -1, bt = -1;
                            if (i0 < q.qlen) { bo = o0; bw = W0; bt = t0; }
                            if (pp1 && k + 1 + o1 < q.qlen && o1 < Lv && (o1 + 1 > bo || (o1 + 1 == bo && W1 + 1 > bw))) {
                                bo = o1 + 1; bw = W1 + 1; bt = t1;
                            }
                            if (pp2 && o2 < Lv && (o2 + 1 > bo || (o2 + 1 == bo && W2 + 1 > bw))) {
                                bo = o2 + 1; bw = W2 + 1; bt = t2;
                            }
                            if (bo >= 0) {
                                if (pp1) {
                                    if (bo > o1) { c2 = bo; cw2 = bw; ct2 = bt; }
                                } else {
                                    c2 = bo; cw2 = bw; ct2 = bt;
                                    rec2 = true;
                                    pg2 = (sl < 31) ? ds0 : dir_insert(q.dir, mask, dkey(v, kp0 + 1), &S.dirn);
                                }
                            }
                        }
                    }
                    // records of the diagonals outside F_s (k-1, k+1), the windows and
                    // v's out-edge record (edge range and first targets, needed when an
                    // output reaches the vertex end), all in one round of loads: every
                    // lane loads every word (one without a use reads a harmless valid
                    // address), so that no load sits in a branch of its own and the
                    // loads are waited for once
                    const int32_t m0 = (c0 >= 0) ? min(q.qlen - (k + c0 - 1), Lv - c0) : 0;
                    const int32_t m1 = (c1 >= 0) ? min(q.qlen - (k + c1), Lv - c1) : 0;
                    const int32_t m2 = (c2 >= 0) ? min(q.qlen - (k + 1 + c2), Lv - c2) : 0;
                    const ull rw0l = q.pages[(rec0 && pg0 >= 0) ? pg0 : 0].R[(k - 1) & 31];
                    const ull rw2l = q.pages[(rec2 && pg2 >= 0) ? pg2 : 0].R[(k + 1) & 31];
                    const int4 vil = vinfo[valid ? v : 0];
                    const ull x0l = win32(q.rd, m0 > 0 ? q.q0 + k - 1 + c0 : q.q0) ^ win32(A.seg, m0 > 0 ? sb + c0 : 0);
                    const ull x1l = win32(q.rd, m1 > 0 ? q.q0 + k + c1 : q.q0) ^ win32(A.seg, m1 > 0 ? sb + c1 : 0);
                    const ull x2l = win32(q.rd, m2 > 0 ? q.q0 + k + 1 + c2 : q.q0) ^ win32(A.seg, m2 > 0 ? sb + c2 : 0);
                    const ull rw0 = (rec0 && pg0 >= 0) ? rw0l : 0ull;
                    const ull rw2 = (rec2 && pg2 >= 0) ? rw2l : 0ull;
                    const int4 vi = valid ? vil : make_int4(0, 0, -1, -1);
                    const ull x0 = (m0 > 0) ? x0l : 0ull;
                    const ull x1 = (m1 > 0) ? x1l : 0ull;
                    const ull x2 = (m2 > 0) ? x2l : 0ull;
                    if (c0 >= 0) {
                        const bool rec = rgen(rw0) == q.gen;
                        if (!rec || c0 > rval(rw0)) {
                            ov0 = true; oo0 = c0; ow0 = W0 + 1; ot0 = t0; od0 = pg0; on0 = !rec;
                        }
                    }
                    if (c1 >= 0) { ov1 = true; oo1 = c1; ow1 = cw1; ot1 = ct1; od1 = ds0; }
                    if (c2 >= 0) {
                        if (!rec2) {
                            ov2 = true; oo2 = c2; ow2 = cw2; ot2 = ct2; od2 = d2; on2 = false;
                        } else {
                            const bool rec = rgen(rw2) == q.gen;
                            if (!rec || c2 > rval(rw2)) { ov2 = true; oo2 = c2; ow2 = cw2; ot2 = ct2; od2 = pg2; on2 = !rec; }
                        }
                    }
                    // extension of the admitted outputs
                    int32_t lx0 = 0, lx1 = 0, lx2 = 0;
                    {
                        chunks += (ov0 && m0 > 0) + (ov1 && m1 > 0) + (ov2 && m2 > 0);
                        lx0 = ov0 ? (x0 ? min((int32_t)(__clzll((long long)x0) >> 1), m0) : min(32, m0)) : 0;
                        lx1 = ov1 ? (x1 ? min((int32_t)(__clzll((long long)x1) >> 1), m1) : min(32, m1)) : 0;
                        lx2 = ov2 ? (x2 ? min((int32_t)(__clzll((long long)x2) >> 1), m2) : min(32, m2)) : 0;
                        // whole windows matched and bases remain: continue (one call
                        // site for the three outputs keeps the register demand down)
#pragma unroll 1
                        for (int j = 0; j < 3; ++j) {
                            const int32_t lj = (j == 0) ? lx0 : ((j == 1) ? lx1 : lx2);
                            const int32_t mj = (j == 0) ? m0 : ((j == 1) ? m1 : m2);
                            if (lj == 32 && mj > 32) {
                                const int32_t oj = (j == 0) ? oo0 : ((j == 1) ? oo1 : oo2);
                                const int32_t r = 32 + lcp<false>(q.rd, q.q0 + k - 1 + j + oj + 32, ((q.q0 + q.qlen) >> 5) + 1, A.seg,
                                                           sb + oj + 32, ((sb + Lv) >> 5) + 1, mj - 32, chunks);
                                if (j == 0) lx0 = r; else if (j == 1) lx1 = r; else lx2 = r;
                            }
                        }
                    }
                    const int cnt = (int)ov0 + (int)ov1 + (int)ov2;
                    int total;
                    const int pos = block_excl_scan<BLOCK>(cnt, total, S.scan);
                    if (base + BLOCK < n) fetch_batch(base + BLOCK);
                    adm += cnt;
                    int slot = 0;
                    int endm = 0;        // outputs that reached the vertex end (cross every out-edge)
                    int deg = 0;
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const bool vj = (j == 0) ? ov0 : ((j == 1) ? ov1 : ov2);
                        if (vj) {
                            const int32_t kj = k - 1 + j;
                            const int32_t lj = (j == 0) ? lx0 : ((j == 1) ? lx1 : lx2);
                            const int32_t o = ((j == 0) ? oo0 : ((j == 1) ? oo1 : oo2)) + lj;
                            const int32_t Wj = ((j == 0) ? ow0 : ((j == 1) ? ow1 : ow2)) + lj;
                            const int32_t tj = (j == 0) ? ot0 : ((j == 1) ? ot1 : ot2);
                            int d = (j == 0) ? od0 : ((j == 1) ? od1 : od2);
                            const bool nw = (j == 0) ? on0 : ((j == 1) ? false : on2);
                            const int32_t p = outbase + pos + slot;
                            ++slot;
                            if (d < 0) d = dir_insert(q.dir, mask, dkey(v, kj >> 5), &S.dirn);
                            if (p >= A.list_cap) {
                                atomicOr(&S.flags, F_LIST);
                            } else if (d < 0) {
                                atomicOr(&S.flags, F_GROW);
                            } else {
                                const int nc = record_entry(q, S, v, kj, o, Wj, d, nw, Lv, o == Lv ? vi.y : 0, lmax);
                                if (nc) { endm |= 1 << j; deg = nc; }
                                Ld.e[p] = make_int4(v, kj, o, d);
                                if ((p & (SAMP - 1)) == 0 && p < SAMP * nsamp(BLOCK)) S.samp[p / SAMP] = skey(v, kj);
                                if (q.track) Ld.w[p] = Wj;
                                if (q.tb) Ld.t[p] = tj;
                            }
                        }
                    }
                    // crossing candidates of the whole wave in one allocation,
                    // skipped when no lane of the wave reached a vertex end
                    if (__ballot(endm != 0)) {
                        const int ncr = __popc(endm) * deg;
                        int cp = wave_alloc(ncr, &S.ncand);
                        if (endm) {
#pragma unroll
                            for (int j = 0; j < 3; ++j) {
                                if (!((endm >> j) & 1)) continue;
                                const int32_t lj = (j == 0) ? lx0 : ((j == 1) ? lx1 : lx2);
                                const int32_t Wj = ((j == 0) ? ow0 : ((j == 1) ? ow1 : ow2)) + lj;
                                const int32_t tj = (j == 0) ? ot0 : ((j == 1) ? ot1 : ot2);
                                const int32_t k2 = k - 1 + j + Lv;
                                put_out_edges(S, A, cu, ck, cW, ct, cp, vi, k2, Wj, tj);
                                cp += deg;
                            }
                        }
                    }
                    outbase += total;
                }
                n1 = min(outbase, A.list_cap);
                if (adm) atomicAdd(&S.adm, (ull)adm);
                if (tid == 0) S.n_out = n1;
            }
            if (tid == 0) { const ull t2 = wall_clock64(); S.tick[0] += t2 - tk; tk = t2; }
            // ========== crossings (Algorithm 2, same score, cost 0), in rounds ==========
            int32_t xlo = n1, xhi = (s == 0) ? n_start : n1;
            const int32_t preset_hi = (s == 0) ? n_start : 0;   // the start entries have their W and t
            bool restart = false;
            for (int round = 0;; ++round) {
                // (1) extend the diagonals created by the previous round
                for (int32_t base = xlo; base < xhi; base += BLOCK) {
                    const int32_t idx = base + tid;
                    int ncr = 0;
                    int32_t k2 = 0, W = 0, t = 0;
                    int4 vi = make_int4(0, 0, -1, -1);
                    if (idx < xhi) {
                        // the entry carries its vertex's label (set when it was claimed),
                        // so the extension's first loads go out with the out-edge range
                        int32_t v, k, d, o, Lv;
                        int64_t sb;
                        if (round > 0 && idx - xlo < SH::XC) {   // claimed by the previous round, at offset 0
                            const int32_t j = idx - xlo;
                            v = S.xsv[j]; k = S.xsk[j]; d = S.xsd[j]; o = 0; Lv = S.xsl[j]; sb = S.xsb[j];
                            t = q.tb ? S.xst[j] : -1;
                        } else {
                            const int4 e = Ld.e[idx];
                            v = e.x; k = e.y; d = e.w; o = e.z;
                            sb = Ld.b[idx];
                            Lv = Ld.l[idx];
                            W = (q.track || idx < preset_hi) ? Ld.w[idx] : 0;
                            t = (q.tb || idx < preset_hi) ? Ld.t[idx] : -1;
                        }
                        if (idx >= preset_hi && q.track) W = rval(q.pages[d].Wc[k & 31]);
                        vi = vinfo[v];
                        // Algorithm 5's push: its map slot is read with the extension's
                        // loads, the push itself follows the extension
                        const bool push = q.tb && idx >= preset_hi;
                        const ull tprobe = __hip_atomic_load(&q.mkey[push ? (dhash(dkey(v, t)) & q.mask) : 0],
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ncr = extend_entry(A, q, S, v, k, o, W, d, true, sb, Lv, vi.y, chunks, lmax);
                        if (idx >= preset_hi) t = push ? trace_push_from(q, S, v, t, tprobe) : -1;
                        Ld.e[idx].z = o;
                        if (q.track) Ld.w[idx] = W;
                        if (q.tb) Ld.t[idx] = t;
                        k2 = k + Lv;
                    }
                    if (__ballot(ncr != 0)) {
                        const int cp = wave_alloc(ncr, &S.ncand);
                        if (ncr) put_out_edges(S, A, cu, ck, cW, ct, cp, vi, k2, W, t);
                    }
                }
                __syncthreads();
                const int32_t nc = __builtin_amdgcn_readfirstlane(S.ncand);
                const int f1 = __builtin_amdgcn_readfirstlane(S.flags | ((S.dirn > half || S.mn > half) ? F_GROW : 0));
                __syncthreads();
                if (tid == 0) S.ncand = 0;
                if (f1) { rflags = f1; restart = true; break; }
                if (nc == 0) break;
                // (2) claim never-seen diagonals (no record of this query); every
                // predecessor of this round folds its W into the slot with a max
                const ull mine = mkR(q.gen, CLAIM_BASE + round);
                for (int32_t base = 0; base < nc; base += BLOCK) {
                    const int32_t c = base + tid;
                    int claim = 0;
                    int ds = -1;
                    int64_t csb = 0;
                    int32_t cLv = 0;
                    int32_t u = 0, kc = 0, wc = 0, tc = -1;
                    if (c < nc) {
                        if (c < SH::CS) {
                            u = S.csu[c]; kc = S.csk[c]; tc = S.cst[c];
                        } else {
                            u = cu[c]; kc = ck[c]; wc = cW[c]; tc = ct[c];
                        }
                        // the target's label (stored with the entry when it is claimed),
                        // the directory slot and the record word in the page of that
                        // slot, read together: the page is almost always at its key's
                        // home slot (found there, or inserted there), and only when it
                        // is not is the record read again from the slot found.  The
                        // early read sees what a later one would: in this phase the
                        // word changes only by the claims' compare-and-swaps, which
                        // compare against the value read.
                        const ull key = dkey(u, kc >> 5);
                        const uint32_t h = dhash(key) & mask;
                        const ull probe = __hip_atomic_load(&q.dir[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const int4 lab = A.vlab[u];
                        const ull wh = __hip_atomic_load(&q.pages[h].R[kc & 31], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                        csb = lab_base(lab);
                        cLv = lab.z;
                        ds = dir_settle(q.dir, mask, key, h, probe, &S.dirn);
                        if (ds < 0) {
                            atomicOr(&S.flags, F_GROW);
                        } else {
                            ull* rp = &q.pages[ds].R[kc & 31];
                            const ull w = (ds == (int)h) ? wh
                                                         : __hip_atomic_load(rp, __ATOMIC_RELAXED,
                                                                             __HIP_MEMORY_SCOPE_AGENT);
                            bool part = false;
                            if (rgen(w) != q.gen) {
                                const ull old = atomicCAS(rp, w, mine);
                                if (old == w) { claim = 1; part = true; }
                                else if (old == mine) part = true;
                            } else if (w == mine) {
                                part = true;
                            }
                            if (part && q.track) atomicMax(&q.pages[ds].Wc[kc & 31], mkR(q.gen, wc));
                        }
                    }
                    const int pos = wave_alloc(claim, &S.n_out);
                    if (claim) {
                        if (pos < A.list_cap) {
                            Ld.e[pos] = make_int4(u, kc, 0, ds);
                            Ld.l[pos] = cLv; Ld.b[pos] = csb;
                            if (q.track) Ld.w[pos] = wc;
                            if (q.tb) Ld.t[pos] = tc;
                            const int32_t j = pos - xhi;
                            if (j < SH::XC) {
                                S.xsv[j] = u; S.xsk[j] = kc; S.xsd[j] = ds; S.xsl[j] = cLv; S.xsb[j] = csb; S.xst[j] = tc;
                            }
                        } else {
                            atomicOr(&S.flags, F_LIST);
                        }
                    }
                }
                __syncthreads();
                const int32_t xn = __builtin_amdgcn_readfirstlane(S.n_out);
                const int f2 = __builtin_amdgcn_readfirstlane(S.flags | ((S.dirn > half) ? F_GROW : 0));
                __syncthreads();
                if (f2) { rflags = f2; restart = true; break; }
                xlo = xhi;
                xhi = xn;
                if (tid == 0) S.cross += (ull)(xhi - xlo);
            }
            if (restart) break;
            if (tid == 0) { const ull t2 = wall_clock64(); S.tick[1] += t2 - tk; tk = t2; }
            const int32_t ntot = xhi;
            work += ntot;
            if (q.track) {   // one update of the score's maxima per wave
                for (int m = 32; m >= 1; m >>= 1) {
                    lmax.x = max(lmax.x, __shfl_xor(lmax.x, m, 64));
                    lmax.y = max(lmax.y, __shfl_xor(lmax.y, m, 64));
                }
                if (__lane_id() == 0) {
                    atomicMax(&S.amax, __builtin_amdgcn_readfirstlane(lmax.x));
                    atomicMax(&S.imax, __builtin_amdgcn_readfirstlane(lmax.y));
                }
            }
            __syncthreads();
            const int found = __builtin_amdgcn_readfirstlane(S.found);
            const int32_t iend = q.ilo < q.qlen ? __builtin_amdgcn_readfirstlane(S.iend) : q.qlen;
            const int32_t amax = __builtin_amdgcn_readfirstlane(S.amax);
            const int32_t imax = __builtin_amdgcn_readfirstlane(S.imax);
            __syncthreads();
            // ========== end test (extension mode) ==========
            if (found) {
                status = GWFA_ST_OK;
                clip = q.qlen - iend;
                if (q.ilo < q.qlen) {
                    // the end cells of row iend (all of them are in this score's list)
                    for (int32_t idx = tid; idx < ntot; idx += BLOCK) {
                        const int4 e = Ld.e[idx];
                        const int32_t v = e.x, o = e.z;
                        if (e.y + o == iend && ends_walk(q, v, o, A.vlab[v].z))
                            atomicMin(&S.endkey, ((ull)(uint32_t)v << 32) | (uint32_t)o);
                    }
                    __syncthreads();
                }
                if (q.tb) {
                    if (tid == 0) S.tend = -1;
                    __syncthreads();
                    const int32_t ev = (int32_t)(S.endkey >> 32), eo = (int32_t)(S.endkey & 0xffffffffull);
                    for (int32_t idx = tid; idx < ntot; idx += BLOCK) {
                        const int4 e = Ld.e[idx];
                        if (e.x == ev && e.z == eo && e.y + eo == iend) S.tend = Ld.t[idx];
                    }
                    __syncthreads();
                }
                break;
            }
            if (A.max_score >= 0 && s >= A.max_score) { status = GWFA_ST_MAX_SCORE; break; }
            // global form: an empty wavefront means the end vertex cannot be
            // reached.  Extension mode: cannot happen for valid input (the
            // query can always be inserted); a guard so that every workgroup
            // finishes.
            if (ntot == 0) { status = q.ve >= 0 ? GWFA_ST_UNREACHABLE : GWFA_ST_MAX_SCORE; break; }
            if (q.ve < 0 && s > q.qlen + 1) { status = GWFA_ST_MAX_SCORE; break; }
            // ========== merge the crossing diagonals into the sorted list ==========
            // Small sets (<= Shared::XS, in lists of up to 32 Shared::XS entries)
            // are merged virtually: their keys are ranked in LDS and each gets
            // its merged position (its rank among the crossing keys plus the
            // number of expansion outputs below it); the next pass reads the list
            // through a bitmap of those positions.  Larger sets are sorted in the
            // arena and the list is rewritten merged.
            const int32_t m = ntot - n1;
            // sampled keys of the expansion's list (none at score 0, where the
            // list is the crossing entries of the start alone)
            const int32_t nsl = s > 0 ? min((int32_t)nsamp(BLOCK), (n1 + SAMP - 1) / SAMP) : 0;
            vmx = 0;
            if (m > 0) {
                if (m > A.sort_cap) { rflags = F_LIST; break; }
                if (m <= SH::XS && ntot <= 32 * SH::XS) {
                    // rank of each crossing key among them (the keys are distinct
                    // diagonals), counted against every key read from LDS by all
                    // lanes at once: two barriers, where a sorting network would
                    // take one per stage
                    for (int i = tid; i < m; i += BLOCK) {
                        const int2 a = vk_of(Ld, n1 + i);
                        S.skeys[i] = skey(a.x, a.y);
                    }
                    __syncthreads();
                    for (int i = tid; i < m; i += BLOCK) {
                        const ull ki = S.skeys[i];
                        int32_t rk = 0;
                        // sixteen keys per step, read together (one LDS round trip per
                        // step instead of one per key)
                        int j = 0;
                        for (; j + 16 <= m; j += 16) {
                            ull x[16];
#pragma unroll
                            for (int u = 0; u < 16; ++u) x[u] = S.skeys[j + u];
#pragma unroll
                            for (int u = 0; u < 16; ++u) rk += x[u] < ki ? 1 : 0;
                        }
                        for (; j < m; ++j) rk += S.skeys[j] < ki ? 1 : 0;
                        S.sidx[rk] = n1 + i;
                        S.xcnt[rk] = rk + lower_bound_sampled(Ld, n1, ki, S.samp, nsl);
                    }
                    __syncthreads();
                    // the merged positions as a bitmap over the list plus the number of
                    // bits below each word, in the keys' storage (no longer needed;
                    // 32 positions per key slot): the passes over this list find an
                    // entry's physical slot from two words
                    {
                        const int32_t nw = (ntot + 31) >> 5;
                        for (int32_t w = tid; w < nw; w += BLOCK) vm_bits[w] = 0u;
                        lds_barrier();
                        for (int32_t j = tid; j < m; j += BLOCK) {
                            const int32_t pj = S.xcnt[j];
                            atomicOr(&vm_bits[pj >> 5], 1u << (pj & 31));
                        }
                        lds_barrier();
                        const int32_t kw = (nw + BLOCK - 1) / BLOCK;   // words per thread, in order
                        const int32_t w0 = min(tid * kw, nw), w1 = min(w0 + kw, nw);
                        int nbits = 0;
                        for (int32_t w = w0; w < w1; ++w) nbits += __popc(vm_bits[w]);
                        int tot;
                        int below = block_excl_scan<BLOCK>(nbits, tot, S.scan);
                        for (int32_t w = w0; w < w1; ++w) {
                            vm_pre[w] = below;
                            below += __popc(vm_bits[w]);
                        }
                        lds_barrier();
                    }
                    vmx = m;
                    cur = nb;
                } else {
                    int N = 1;
                    while (N < m) N <<= 1;
                    if (N > A.sort_cap) { rflags = F_LIST; break; }
                    for (int i = tid; i < N; i += BLOCK) {
                        ull key = ~0ull;
                        if (i < m) {
                            const int2 a = vk_of(Ld, n1 + i);
                            key = skey(a.x, a.y);
                        }
                        gkeys[i] = key;
                        gidx[i] = n1 + i;
                    }
                    __syncthreads();
                    bitonic<BLOCK, false>(gkeys, gidx, N);
                    const Lists Lm = LL(cur);
                    for (int32_t j = tid; j < n1; j += BLOCK) {
                        const int2 a = vk_of(Ld, j);
                        copy_entry(Ld, j, Lm, j + lower_bound_keys(gkeys, m, skey(a.x, a.y)), q.track, q.tb);
                    }
                    for (int32_t x = tid; x < m; x += BLOCK)
                        copy_entry(Ld, gidx[x], Lm, x + lower_bound_sampled(Ld, n1, gkeys[x], S.samp, nsl), q.track,
                                   q.tb);
                    __syncthreads();
                }
            } else {
                cur = nb;
            }
            if (tid == 0) { const ull t2 = wall_clock64(); S.tick[2] += t2 - tk; tk = t2; }
            n_cur = ntot;
            // ========== pruning (Algorithm 4) ==========
            if ((MODE == 1 || MODE == 2) && A.prune == GWFA_PRUNE_HEURISTIC && amax > A.a_diff) {
                const Lists Ls = LL(cur);
                const Lists Lp = LL(1 - cur);
                int32_t outbase = 0;
                int dropped = 0;
                for (int32_t base = 0; base < n_cur; base += BLOCK) {
                    const int32_t idx = base + tid;
                    int keep = 0;
                    int32_t ph = idx;
                    if (idx < n_cur) {
                        if (vmx) ph = vm_phys_bm(vm_bits, vm_pre, S.sidx, idx);
                        const int4 e = Ls.e[ph];
                        const int32_t a = e.y + e.z + Ls.w[ph];
                        keep = (amax - a < A.a_diff) ? 1 : 0;
                        if (!keep) {   // the diagonal keeps its offset as its record
                            q.pages[e.w].R[e.y & 31] = mkR(q.gen, e.z);
                            ++dropped;
                        }
                    }
                    int total;
                    const int pos = block_excl_scan<BLOCK>(keep, total, S.scan);
                    if (keep) copy_entry(Ls, ph, Lp, outbase + pos, q.track, q.tb);
                    outbase += total;
                }
                if (dropped) atomicAdd(&S.dropped, dropped);
                cur = 1 - cur;
                n_cur = outbase;
                vmx = 0;
                __syncthreads();
                if (tid == 0) S.tick[3] += wall_clock64() - tk;
            }
            // ========== trace dump and learned keep/drop ==========
            const bool run_mlp = LEARN && A.prune == GWFA_PRUNE_LEARNED && n_cur >= A.mlp_gate && (s % A.mlp_period) == 0;
            if (LEARN && ((DUMP && A.dump) || run_mlp)) {
                const Lists Ls = LL(cur);
                const Lists Lp = LL(1 - cur);
                int32_t outbase = 0;
                int dropped = 0, evals = 0;
                for (int32_t base = 0; base < n_cur; base += BLOCK) {
                    const int32_t idx = base + tid;
                    const bool live = idx < n_cur;
                    int keep = 0;
                    int32_t ph = idx;
                    int rec = 0;
                    float f[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    int32_t v = 0, k = 0, o = 0, dp = 0, W = 0, i = 0;
                    if (live) {
                        if (vmx) ph = vm_phys_bm(vm_bits, vm_pre, S.sidx, idx);
                        const int4 e = Ls.e[ph];
                        v = e.x; k = e.y; o = e.z; dp = e.w; W = Ls.w[ph];
                        i = k + o;
                        const int32_t Lv = A.vlab[v].z;
                        entry_features(f, s, i, W, o, Lv, vinfo[v].y, amax, imax, q.qlen);
                        rec = (DUMP && A.dump) ? 1 : 0;
                        keep = 1;
                    }
                    if (run_mlp) {
                        // the whole wave scores its 64 entries together (matrix cores)
                        const float z = mlp_logit_wave(f, S.mscale, S.mlpw);
                        if (live) {
                            ++evals;
                            keep = (z >= A.keep_threshold || i + W == amax) ? 1 : 0;   // the furthest diagonal stays
                            if (!keep) {
                                q.pages[dp].R[k & 31] = mkR(q.gen, o);   // record kept, as in Algorithm 4
                                ++dropped;
                            }
                        }
                    }
                    if (DUMP && A.dump) {
                        // one global atomic per wave
                        int tot;
                        const int ex = wave_excl_scan(rec, tot);
                        ull b0 = 0;
                        if (__lane_id() == 0 && tot > 0) b0 = atomicAdd(A.dump_count, (ull)tot);
                        b0 = __shfl(b0, 0, 64);
                        const ull slot = b0 + (ull)ex;
                        if (rec && (int64_t)slot < A.dump_cap) {
                            float* dr = A.dump + slot * 16;
#pragma unroll
                            for (int j = 0; j < 8; ++j) dr[j] = f[j];
                            int32_t* di = reinterpret_cast<int32_t*>(dr + 8);
                            di[0] = r; di[1] = s; di[2] = i; di[3] = v; di[4] = o; di[5] = W; di[6] = k;
                            di[7] = (A.tier << 8) | cap_log2;   // attempt: later attempts of a query supersede
                        }
                    }
                    if (run_mlp) {
                        int total;
                        const int pos = block_excl_scan<BLOCK>(keep, total, S.scan);
                        if (keep) copy_entry(Ls, ph, Lp, outbase + pos, q.track, q.tb);
                        outbase += total;
                    }
                }
                if (run_mlp) {
                    if (dropped) atomicAdd(&S.dropped, dropped);
                    if (evals) atomicAdd(&S.mlp, (ull)evals);
                    cur = 1 - cur;
                    n_cur = outbase;
                    vmx = 0;
                }
                __syncthreads();
            }
        }
        if (status >= 0 || !(rflags)) break;
        // capacity exceeded: grow the directory if possible, else give up
        __syncthreads();
        if ((rflags & F_GROW) && !(rflags & F_LIST) && cap_log2 < A.dir_log2_max) {
            cap_log2 = min(cap_log2 + 2, A.dir_log2_max);
            continue;
        }
        status = GWFA_ST_ARENA;
        break;
    }
    if (chunks) atomicAdd(&S.chunks, (ull)chunks);
    __syncthreads();
    // ========== results and walk (Algorithm 6) ==========
    if (tid == 0) {
        out->t_begin = t_begin;
        out->t_end = (int64_t)wall_clock64();
        out->status = status;
        out->n_scores = s + 1;
        out->work = work;
        out->path_off = -1;
        out->path_len = 0;
        out->start_off = q.j0;
        out->clip = clip;
        if (status == GWFA_ST_OK) {
            out->dist = s;
            out->end_v = (int32_t)(S.endkey >> 32);
            out->end_off = (int32_t)(S.endkey & 0xffffffffull);
            if (q.tb && S.tend >= 0) {
                // a chain visits each trace slot at most once: at most mask+1 steps
                const int32_t lim = (int32_t)q.mask + 1;
                int32_t len = 0, first = -1;
                for (int32_t t = S.tend; t >= 0 && len <= lim; t = q.Tt[t]) { ++len; first = t; }
                // the first record's predecessor field holds -1 - (start offset)
                if (first >= 0 && q.Tt[first] < 0) out->start_off = -1 - q.Tt[first];
                const ull pos = atomicAdd(A.path_cursor, (ull)len);
                out->path_len = len;
                if ((int64_t)pos + len <= A.path_cap && A.path_buf) {
                    int32_t j = len - 1;
                    for (int32_t t = S.tend; t >= 0 && j >= 0; t = q.Tt[t]) A.path_buf[pos + (j--)] = q.Tv[t];
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
            atomicAdd(&A.stats[8], (ull)(s + 1));
            for (int i = 0; i < 4; ++i) atomicAdd(&A.stats[9 + i], S.tick[i]);
        }
    }
    __syncthreads();
}

// Waves per SIMD the compiler must allow: 3 (168 registers), 2 for the dump
// instantiation; a 512-lane workgroup fills a CU alone: it takes the whole
// register file instead of spilling.
template <int BLOCK, int MODE>
__global__ __launch_bounds__(BLOCK, MODE == 2 ? 2 : (BLOCK >= 512 ? (MODE == 0 ? 4 : 1) : (MODE == 3 ? 3 : 4))) void k_align(KArgs A) {
    constexpr bool LEARN = MODE >= 2;
    __shared__ Shared<BLOCK, MODE> S;
    char* arena = A.arena + (int64_t)blockIdx.x * A.arena_stride;
    if constexpr (LEARN) {
        if (A.prune == GWFA_PRUNE_LEARNED) {
            for (int i = threadIdx.x; i < MLP_N; i += BLOCK) S.mlpw[i] = A.mlp_w[i];
            if (threadIdx.x < 8) S.mscale[threadIdx.x] = A.mlp_scale[threadIdx.x];
            __syncthreads();
        }
    }
    // queries to take: those the screen pass listed, or all of `order`
    const int32_t n_q = A.n_valid ? __builtin_amdgcn_readfirstlane(*A.n_valid) : A.n_reads;
    for (;;) {
        if (threadIdx.x == 0) S.read = atomicAdd(A.queue, 1);
        __syncthreads();
        const int ridx = __builtin_amdgcn_readfirstlane(S.read);
        __syncthreads();
        if (ridx >= n_q) break;
        const int r = A.order ? A.order[ridx] : ridx;
        align_read<BLOCK, MODE>(A, arena, r, S);
    }
}

// Screen pass (one workgroup, before the alignment kernel): a query whose
// start vertex, start window (0 <= j0 <= j1 <= |v_s|) or end vertex is out
// of range gets its result here, with status GWFA_ST_BAD_INPUT; the others
// are listed in `valid` in the work-queue order (an ordered block scan per
// chunk of SCREEN queries), so that the alignment kernel only ever takes
// queries whose parameters index the graph in bounds.
constexpr int SCREEN = 1024;
__global__ __launch_bounds__(SCREEN) void k_screen(KArgs A, int32_t* valid, int32_t* n_valid) {
    __shared__ int32_t wsum[SCREEN / 64];
    __shared__ int32_t base;
    const int tid = threadIdx.x;
    if (tid == 0) base = 0;
    __syncthreads();
    for (int32_t c = 0; c < A.n_reads; c += SCREEN) {
        const int32_t idx = c + tid;
        int ok = 0;
        int32_t r = 0;
        if (idx < A.n_reads) {
            r = A.order ? A.order[idx] : idx;
            const int32_t vs = A.v_start[r];
            const int32_t ve = A.v_end ? A.v_end[r] : A.end_vertex;
            const int32_t j0 = A.v_off ? A.v_off[r] : 0;
            const int32_t j1 = A.v_off_hi ? A.v_off_hi[r] : j0;
            bool good = vs >= 0 && vs < A.n_vtx && ve >= -1 && ve < A.n_vtx && !(A.v_end && ve < 0) && j0 >= 0 &&
                        j1 >= j0;
            if (good) good = (int64_t)j1 <= A.seg_off[vs + 1] - A.seg_off[vs];
            ok = good ? 1 : 0;
            if (!good) {
                gwfa_result* out = A.res + r;
                const int64_t t = (int64_t)wall_clock64();
                out->t_begin = t; out->t_end = t;
                out->dist = -1; out->end_v = -1; out->end_off = -1; out->status = GWFA_ST_BAD_INPUT;
                out->path_off = -1; out->path_len = 0; out->n_scores = 0; out->work = 0;
                out->start_off = j0; out->clip = 0;
            }
        }
        // ordered exclusive scan of ok over the block
        const ull m = __ballot(ok);
        const int ex = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (__lane_id() == 0) wsum[tid >> 6] = __popcll(m);
        __syncthreads();
        int before = base, tot = 0;
        for (int w = 0; w < SCREEN / 64; ++w) {
            const int x = wsum[w];
            before += (w < (tid >> 6)) ? x : 0;
            tot += x;
        }
        if (ok) valid[before + ex] = r;
        __syncthreads();
        if (tid == 0) base += tot;
        __syncthreads();
    }
    if (tid == 0) *n_valid = base;
}

// Four ASCII bases (the first in the low byte) -> 8 bits, the first base in
// the high bits; A/a 0, C/c 1, G/g 2, T/t 3 come from bits 1-2 of the code
// point ((c >> 1) ^ (c >> 2)).  *bad gets a bit for every other byte.
__device__ __forceinline__ uint32_t pack4(uint32_t x, uint32_t& bad) {
    const uint32_t u = x & 0xDFDFDFDFu;   // upper case
    // 0x80 in every zero byte of v (exact: no carry crosses a byte)
    auto zb = [](uint32_t v) { return ~(((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v | 0x7F7F7F7Fu); };
    const uint32_t ok = zb(u ^ 0x41414141u) | zb(u ^ 0x43434343u) | zb(u ^ 0x47474747u) | zb(u ^ 0x54545454u);
    bad |= ok ^ 0x80808080u;
    const uint32_t m = ((x >> 1) ^ (x >> 2)) & 0x03030303u;
    return ((m & 0xFFu) << 6) | (((m >> 8) & 0xFFu) << 4) | (((m >> 16) & 0xFFu) << 2) | (m >> 24);
}

// ASCII -> 2-bit packed words.  One thread per 16 bases (one 16-byte load,
// so a wave reads 1 KiB contiguously); lane pairs join their halves into one
// 64-bit word (the even lane holds the first 16 bases).
__global__ void k_pack(const uint8_t* __restrict__ ascii, int64_t n, ull* __restrict__ out, int64_t n_words,
                       int32_t* err) {
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b0 = h * 16;
    uint32_t half = 0, bad = 0;
    if (h < 2 * n_words) {
        if (b0 + 16 <= n && ((reinterpret_cast<uintptr_t>(ascii + b0) & 15) == 0)) {
            const uint4 x = *reinterpret_cast<const uint4*>(ascii + b0);
            half = (pack4(x.x, bad) << 24) | (pack4(x.y, bad) << 16) | (pack4(x.z, bad) << 8) | pack4(x.w, bad);
        } else {
            for (int j = 0; j < 16; ++j) {
                const int64_t bi = b0 + j;
                uint32_t code = 0;
                if (bi < n) {
                    const uint32_t c = ascii[bi];
                    const uint32_t u = c & 0xdfu;
                    bad |= (u != 'A' && u != 'C' && u != 'G' && u != 'T');
                    code = ((c >> 1) ^ (c >> 2)) & 3u;
                }
                half = (half << 2) | code;
            }
        }
    }
    // every lane takes part in the exchange (blocks are whole waves, and lane
    // pairs never straddle a wave)
    const uint32_t other = __shfl_xor(half, 1, 64);
    if (h < 2 * n_words && (h & 1) == 0) out[h >> 1] = ((ull)half << 32) | other;
    if (bad && err) atomicExch(err, (int32_t)GWFA_ERR_ALPHABET);
}

// Working memory of the entry point that allocates nothing: one copy per
// device, held from the library's first use on that device to the end of the
// process.  Host code never names it directly (there it is only a stand-in
// for the device symbol): gwfa_static_scratch looks its address up.
static __device__ __align__(256) unsigned char scratch[STATIC_BYTES];

__global__ void k_zero(ull* p, int64_t n_words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void k_reset(int32_t* queue, ull* path_cursor, int32_t* retry_count, ull* dump_count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *queue = 0;
        if (path_cursor) *path_cursor = 0;
        if (retry_count) *retry_count = 0;
        if (dump_count) *dump_count = 0;
    }
}

}  // namespace gwfa_dev

// ---------------------------------------------------------------------------
// launch helpers (called from the host code)
// ---------------------------------------------------------------------------
namespace {
template <int L>
void launch_modes(const KArgs& A, int mode, int groups, hipStream_t st) {
    if (mode == 3) { hipLaunchKernelGGL((gwfa_dev::k_align<L, 3>), dim3(groups), dim3(L), 0, st, A); return; }
    if (mode == 2) { hipLaunchKernelGGL((gwfa_dev::k_align<L, 2>), dim3(groups), dim3(L), 0, st, A); return; }
    if (mode == 1) hipLaunchKernelGGL((gwfa_dev::k_align<L, 1>), dim3(groups), dim3(L), 0, st, A);
    else hipLaunchKernelGGL((gwfa_dev::k_align<L, 0>), dim3(groups), dim3(L), 0, st, A);
}
}  // namespace

hipError_t gwfa_launch_align(const KArgs& A, int lanes, int groups, hipStream_t st) {
    // the trace dump and the learned keep/drop live in their own instantiations
    const int mode = A.dump != nullptr ? 2
                     : (A.prune == GWFA_PRUNE_LEARNED ? 3 : (A.prune != GWFA_PRUNE_NONE ? 1 : 0));
    (void)hipGetLastError();   // the launch status below must not report an older, unrelated error
    switch (lanes) {
    case 64: launch_modes<64>(A, mode, groups, st); break;
    case 128: launch_modes<128>(A, mode, groups, st); break;
    case 256: launch_modes<256>(A, mode, groups, st); break;
    case 512: launch_modes<512>(A, mode, groups, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int gwfa_align_blocks_per_cu(int lanes) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (lanes) {
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gwfa_dev::k_align<64, 0>, 64, 0); break;
    case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gwfa_dev::k_align<128, 0>, 128, 0); break;
    case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gwfa_dev::k_align<256, 0>, 256, 0); break;
    case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gwfa_dev::k_align<512, 0>, 512, 0); break;
    default: break;
    }
    return (e == hipSuccess && nb > 0) ? nb : 0;
}

hipError_t gwfa_launch_pack(const uint8_t* ascii, int64_t n, unsigned long long* out, int64_t n_words, int32_t* err,
                            hipStream_t st) {
    if (n_words <= 0) return hipSuccess;
    const int tpb = 256;
    const int64_t blocks = (2 * n_words + tpb - 1) / tpb;   // one thread per 16 bases
    (void)hipGetLastError();
    hipLaunchKernelGGL(gwfa_dev::k_pack, dim3((unsigned)blocks), dim3(tpb), 0, st, ascii, n, out, n_words, err);
    return hipGetLastError();
}

void* gwfa_static_scratch(int device) {
    static std::mutex mu;
    static void* ptr[64] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0 || device >= 64) return nullptr;
    if (ptr[device]) return ptr[device];
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(gwfa_dev::scratch)) != hipSuccess || !p) return nullptr;
    // generation 0 everywhere (record words of generation 0 read as "never
    // seen"); done once, before any alignment on this device uses it
    (void)hipGetLastError();
    hipLaunchKernelGGL(gwfa_dev::k_zero, dim3(2048), dim3(256), 0, nullptr, (unsigned long long*)p, STATIC_BYTES / 8);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return nullptr;
    ptr[device] = p;
    return p;
}

hipError_t gwfa_launch_screen(const KArgs& A, int32_t* valid, int32_t* n_valid, hipStream_t st) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(gwfa_dev::k_screen, dim3(1), dim3(gwfa_dev::SCREEN), 0, st, A, valid, n_valid);
    return hipGetLastError();
}

hipError_t gwfa_launch_reset(int32_t* queue, unsigned long long* cursor, int32_t* retry_count,
                             unsigned long long* dump_count, hipStream_t st) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(gwfa_dev::k_reset, dim3(1), dim3(64), 0, st, queue, cursor, retry_count, dump_count);
    return hipGetLastError();
}
