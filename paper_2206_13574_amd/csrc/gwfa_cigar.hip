// gwfa_cigar.hip -- base-level alignment of each query against the walk the
// graph alignment traced (the last step the paper leaves to a pairwise
// aligner, noting that it is cheap).
//
// One persistent workgroup per query: the walk's string T (the labels of the
// walk, the first one from start_off, the last one cut at end_off) is
// spelled into a 2-bit packed buffer,
// then a pairwise wavefront alignment (the score-ordered diagonal recurrence
// of Eq. 2 on a single path: mismatch, insertion, deletion, then extension
// by the exact-match run) finds an optimal global alignment of q and T, and
// one thread walks the stored wavefronts back into CIGAR operations.
//
// Wavefront s covers diagonals k = j - i in [-s, s] (i query bases, j bases
// of T consumed) and is stored at offset s*s of the workgroup's buffer, so a
// distance d needs (d+1)^2 words.  Operation words are (length << 4) | op
// with op 7 ('=', match), 8 ('X', mismatch), 1 ('I', query base absent from
// the walk), 2 ('D', walk base absent from the query), 4 ('S', query bases
// left unaligned by a free end gap in the query), as in SAM/BAM.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gwfa_internal.h"

namespace gwfa_cig {

typedef unsigned long long ull;
constexpr int32_t NEG = -(1 << 30);
constexpr uint32_t OP_EQ = 7, OP_X = 8, OP_I = 1, OP_D = 2, OP_S = 4;

__device__ __forceinline__ ull win32(const ull* __restrict__ w, int64_t p) {
    const int64_t wi = p >> 5;
    const int sh = (int)(p & 31) * 2;
    return (w[wi] << sh) | ((w[wi + 1] >> 1) >> (63 - sh));
}

// exact-match run of q[qp ...] and t[tp ...], at most lim bases, 32 at a time
__device__ int32_t run_len(const ull* __restrict__ q, int64_t qp, const ull* __restrict__ t, int64_t tp, int32_t lim) {
    int32_t l = 0;
    while (l < lim) {
        const ull x = win32(q, qp + l) ^ win32(t, tp + l);
        const int32_t m = x ? (int32_t)(__clzll((long long)x) >> 1) : 32;
        if (l + m >= lim) return lim;
        l += m;
        if (x) return l;
    }
    return l;
}

// the three sources of diagonal k at score s (Eq. 2 on one path); NEG if absent
__device__ __forceinline__ void sources(const int32_t* __restrict__ Wp, int32_t sp, int32_t k, int32_t qlen,
                                        int32_t tlen, int32_t& mis, int32_t& ins, int32_t& del) {
    mis = ins = del = NEG;
    if (k >= -sp && k <= sp) {                    // mismatch: (i, j) -> (i+1, j+1)
        const int32_t i0 = Wp[k + sp];
        if (i0 >= 0 && i0 < qlen && i0 + k < tlen) mis = i0 + 1;
    }
    if (k + 1 >= -sp && k + 1 <= sp) {            // query base alone: (i, j) -> (i+1, j), from k+1
        const int32_t i1 = Wp[k + 1 + sp];
        if (i1 >= 0 && i1 < qlen) ins = i1 + 1;
    }
    if (k - 1 >= -sp && k - 1 <= sp) {            // walk base alone: (i, j) -> (i, j+1), from k-1
        const int32_t i2 = Wp[k - 1 + sp];
        if (i2 >= 0 && i2 + k - 1 < tlen) del = i2;
    }
}

struct Shared {
    int32_t read;
    int32_t done;
    int32_t scan[16];
    int64_t carry;
};

// The query's result as scalars: every field is read by one lane and
// broadcast, so that every branch on it is a branch of the whole workgroup.
struct UniRes {
    int32_t dist, end_off, status, path_len, start_off, clip;
    int64_t path_off;
};
__device__ __forceinline__ int64_t uni64(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ UniRes load_res(const gwfa_result* p) {
    UniRes u;
    u.dist = __builtin_amdgcn_readfirstlane(p->dist);
    u.end_off = __builtin_amdgcn_readfirstlane(p->end_off);
    u.status = __builtin_amdgcn_readfirstlane(p->status);
    u.path_len = __builtin_amdgcn_readfirstlane(p->path_len);
    u.start_off = __builtin_amdgcn_readfirstlane(p->start_off);
    u.clip = __builtin_amdgcn_readfirstlane(p->clip);
    u.path_off = uni64(p->path_off);
    return u;
}

// Persistent loop over the queries.  No query leaves the loop body early
// (no continue, no return): a per-query exit in front of the queue fetch
// (thread 0's atomic, then a barrier) lets the compiler send the other lanes
// straight back to that barrier while thread 0 waits outside the loop, and
// the workgroup never fetches again.  Every branch that decides the loop's
// course is on values the whole workgroup shares (scalar registers).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_cigar(CigArgs A) {
    __shared__ Shared S;
    char* arena = A.arena + (int64_t)blockIdx.x * A.arena_stride;
    ull* T = reinterpret_cast<ull*>(arena);
    int64_t* P = reinterpret_cast<int64_t*>(arena + A.o_pref);
    int32_t* W = reinterpret_cast<int32_t*>(arena + A.o_wf);
    uint32_t* ops = reinterpret_cast<uint32_t*>(arena + A.o_ops);
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) S.read = atomicAdd(A.queue, 1);
        __syncthreads();
        const int r = __builtin_amdgcn_readfirstlane(S.read);
        __syncthreads();
        if (r >= A.n_reads) break;
        const UniRes res = load_res(A.res + r);
        const int64_t q0 = uni64(A.rd_off[r]);
        const int32_t qfull = __builtin_amdgcn_readfirstlane((int32_t)(A.rd_off[r + 1] - q0));
        // the graph alignment covers q[0, qfull - clip); the rest is soft-clipped
        const int32_t qlen = qfull - res.clip;
        const bool usable = res.status == GWFA_ST_OK && res.path_off >= 0 && res.path_len > 0 &&
                            res.dist <= A.max_d && qfull <= A.max_q && res.start_off >= 0 && res.clip >= 0 &&
                            qlen >= 0;
        if (!usable) {
            if (tid == 0) { A.cigar_off[r] = -1; A.cigar_len[r] = -1; }
        } else {
            const int32_t* walk = A.path_buf + res.path_off;
            const int32_t L = res.path_len;
            const int32_t j0 = res.start_off;
            // ---- prefix offsets of the walk's vertices in T (block scan in chunks)
            if (tid == 0) S.carry = 0;
            __syncthreads();
            for (int32_t b = 0; b < L; b += BLOCK) {
                const int32_t j = b + tid;
                int64_t len = 0;
                if (j < L) {
                    const int32_t v = walk[j];
                    len = (j == L - 1) ? (int64_t)res.end_off : (A.seg_off[v + 1] - A.seg_off[v]);
                    if (j == 0) len = max(len - j0, (int64_t)0);   // the first vertex starts at j0
                }
                // inclusive scan over the block (the lengths fit in 32 bits per vertex)
                int32_t x = (int32_t)len;
                for (int d = 1; d < 64; d <<= 1) {
                    const int32_t y = __shfl_up(x, d, 64);
                    if (__lane_id() >= d) x += y;
                }
                if (__lane_id() == 63) S.scan[tid >> 6] = x;
                __syncthreads();
                int64_t before = S.carry;
                for (int w = 0; w < (tid >> 6); ++w) before += S.scan[w];
                if (j < L) P[j + 1] = before + x;
                if (j == 0) P[0] = 0;
                __syncthreads();
                if (tid == 0) {
                    int64_t tot = 0;
                    for (int w = 0; w < BLOCK / 64; ++w) tot += S.scan[w];
                    S.carry += tot;
                }
                __syncthreads();
            }
            const int64_t tlen64 = uni64(S.carry);
            if (tlen64 > (int64_t)A.max_t) {
                if (tid == 0) { A.cigar_off[r] = -1; A.cigar_len[r] = -3; }
            } else {
                const int32_t tlen = (int32_t)tlen64;
                // ---- spell T, 2-bit packed, 32 bases per word, plus two zero words
                const int32_t tw = tlen / 32 + 2;
                for (int32_t w = tid; w < tw; w += BLOCK) {
                    ull word = 0;
                    int64_t p = (int64_t)w * 32;
                    if (p < tlen) {
                        int32_t lo = 0, hi = L - 1;          // last vertex j with P[j] <= p
                        while (lo < hi) {
                            const int32_t mid = (lo + hi + 1) >> 1;
                            if (P[mid] <= p) lo = mid; else hi = mid - 1;
                        }
                        int32_t j = lo;
                        for (int b = 0; b < 32 && p < tlen; ++b, ++p) {
                            while (j + 1 < L && P[j + 1] <= p) ++j;
                            const int64_t g = A.seg_off[walk[j]] + (j == 0 ? j0 : 0) + (p - P[j]);
                            const ull c = (A.seg[g >> 5] >> (62 - 2 * (g & 31))) & 3ull;
                            word |= c << (62 - 2 * b);
                        }
                    }
                    T[w] = word;
                }
                __syncthreads();
                // ---- wavefronts
                const int32_t kend = tlen - qlen;
                if (tid == 0) {
                    const int32_t l = run_len(A.rd, q0, T, 0, min(qlen, tlen));
                    W[0] = l;
                    S.done = (kend == 0 && l == qlen) ? 0 : -1;
                }
                __syncthreads();
                int32_t done = __builtin_amdgcn_readfirstlane(S.done);
                __syncthreads();
                int32_t s = 0;
                while (done < 0 && s < A.max_d) {
                    ++s;
                    const int32_t* Wp = W + (int64_t)(s - 1) * (s - 1);
                    int32_t* Ws = W + (int64_t)s * s;
                    for (int32_t k = -s + tid; k <= s; k += BLOCK) {
                        int32_t mis, ins, del;
                        sources(Wp, s - 1, k, qlen, tlen, mis, ins, del);
                        int32_t i = max(mis, max(ins, del));
                        if (i >= 0) i += run_len(A.rd, q0 + i, T, (int64_t)i + k, min(qlen - i, tlen - i - k));
                        Ws[k + s] = i < 0 ? NEG : i;
                        if (k == kend && i == qlen) S.done = s;
                    }
                    // every thread reads the flag between two barriers, so all take
                    // the same decision before anyone can set it again
                    __syncthreads();
                    done = __builtin_amdgcn_readfirstlane(S.done);
                    __syncthreads();
                }
                const int32_t dd = done;
                if (tid == 0) {
                    if (dd < 0) {
                        A.cigar_off[r] = -1;
                        A.cigar_len[r] = -3;
                    } else {
                        // ---- traceback: operations from the end, run-length merged
                        int32_t n = 0;
                        auto emit = [&](uint32_t op, int32_t len) {
                            if (len <= 0) return;
                            if (n > 0 && (ops[n - 1] & 15u) == op) ops[n - 1] += (uint32_t)len << 4;
                            else ops[n++] = ((uint32_t)len << 4) | op;
                        };
                        emit(OP_S, qfull - qlen);
                        int32_t k = kend, i = qlen;
                        for (int32_t ss = dd; ss > 0; --ss) {
                            int32_t mis, ins, del;
                            sources(W + (int64_t)(ss - 1) * (ss - 1), ss - 1, k, qlen, tlen, mis, ins, del);
                            const int32_t v = max(mis, max(ins, del));
                            emit(OP_EQ, i - v);
                            if (mis == v) { emit(OP_X, 1); i = v - 1; }
                            else if (ins == v) { emit(OP_I, 1); i = v - 1; k += 1; }
                            else { emit(OP_D, 1); i = v; k -= 1; }
                        }
                        emit(OP_EQ, i);
                        // reverse into the output
                        const ull pos = atomicAdd(A.cigar_cursor, (ull)n);
                        if ((int64_t)pos + n <= A.cigar_cap) {
                            for (int32_t x = 0; x < n; ++x) A.cigar[pos + x] = ops[n - 1 - x];
                            A.cigar_off[r] = (int64_t)pos;
                            A.cigar_len[r] = n;
                        } else {
                            A.cigar_off[r] = -1;
                            A.cigar_len[r] = -2;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

__global__ void k_cig_reset(int32_t* queue, ull* cursor) {
    if (threadIdx.x == 0 && blockIdx.x == 0) { *queue = 0; *cursor = 0; }
}

}  // namespace gwfa_cig

hipError_t gwfa_launch_cigar(const CigArgs& A, int groups, hipStream_t st) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(gwfa_cig::k_cig_reset, dim3(1), dim3(64), 0, st, A.queue, A.cigar_cursor);
    hipLaunchKernelGGL(gwfa_cig::k_cigar<256>, dim3(groups), dim3(256), 0, st, A);
    return hipGetLastError();
}
