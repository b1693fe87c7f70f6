// gwfa_internal.h -- launch arguments shared by the host code and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gwfa.h"

struct KArgs {
    // graph (device)
    const unsigned long long* seg;   // packed labels
    const int64_t* seg_off;          // n_vtx+1 base offsets
    const int32_t* out_off;          // n_vtx+1 CSR offsets
    const int32_t* out_dst;          // n_edge targets
    const int4* vinfo;               // n_vtx: first out-edge index, out-degree, first and second target (-1: none)
    const int4* vlab;                // n_vtx: label base (low, high 32 bits), label length, 0
    int32_t n_vtx;
    // queries (device)
    const unsigned long long* rd;    // packed queries
    const int64_t* rd_off;           // n_reads+1 base offsets
    const int32_t* v_start;
    const int32_t* v_off;            // per-query start offsets in the start vertex, or null (all 0)
    const int32_t* v_off_hi;         // per-query end of a free start window, or null (= v_off)
    const int32_t* order;            // work-queue order or null
    const int32_t* n_valid;          // queries in `order` (written by the screen pass), or null: n_reads
    const int32_t* v_end;            // per-query end vertices (global form) or null
    int32_t end_vertex;              // end vertex of every query (global form) or -1
    int32_t n_reads;
    // outputs (device)
    gwfa_result* res;
    int32_t* path_buf;
    int64_t path_cap;
    unsigned long long* path_cursor;
    int32_t* queue;
    unsigned long long* stats;       // 8 counters or null
    int32_t* retry;                  // queries that overflowed (or null)
    int32_t* retry_count;
    // options
    int32_t prune, a_diff, traceback, max_score;
    float keep_threshold;
    int32_t mlp_gate, mlp_period;
    int32_t end_free;                // free end gap in the query (trailing bases)
    int32_t walk_free;               // global form: the walk may end anywhere inside the end vertex
    const uint16_t* mlp_w;           // bf16 weights (device) or null
    const float* mlp_scale;          // 8 feature scales (device) or null
    float* dump;                     // per-entry trace records (16 x 4 bytes) or null
    int64_t dump_cap;
    unsigned long long* dump_count;
    int32_t tier;                    // working-memory tier of this launch (tags dump records)
    // working memory: one arena per workgroup
    char* arena;
    int64_t arena_stride;
    int32_t dir_log2_max, dir_factor, list_cap, cand_cap, sort_cap;
    int64_t o_hdr, o_dir, o_pages, o_mkey, o_tv, o_tt, o_lists, o_cand, o_sort;
};

hipError_t gwfa_launch_align(const KArgs& A, int lanes, int groups, hipStream_t st);
// resident workgroups per compute unit of the exact alignment kernel (0 if unknown)
int gwfa_align_blocks_per_cu(int lanes);
hipError_t gwfa_launch_pack(const uint8_t* ascii, int64_t n, unsigned long long* out, int64_t n_words,
                            int32_t* err, hipStream_t st);
hipError_t gwfa_launch_reset(int32_t* queue, unsigned long long* cursor, int32_t* retry_count,
                             unsigned long long* dump_count, hipStream_t st);
// Working memory of the entry point that allocates nothing
// (gwfa_align_batch_static_dev): a file-scope device array of STATIC_BYTES
// per device holding a header (queue, counters), the screened query list
// (at most STATIC_MAX_READS queries) and one fixed tier of per-workgroup
// arenas (record directory of 2^STATIC_DIR_LOG2 pages, wavefront lists of
// STATIC_LIST_CAP entries).
constexpr int64_t STATIC_BYTES = (int64_t)512 << 20;
constexpr int32_t STATIC_MAX_READS = 1 << 20;
constexpr int32_t STATIC_DIR_LOG2 = 14;
constexpr int32_t STATIC_LIST_CAP = 8192;
constexpr int64_t STATIC_HDR = 4096;   // queue, retry counter, screened count, path cursor
// Device address of the static array on `device` (the current device),
// looked up and cleared once per device and process; null if that fails.
void* gwfa_static_scratch(int device);

// per-query parameter check before the alignment: results of the queries
// that are out of range (GWFA_ST_BAD_INPUT), the others listed in `valid`
// in work-queue order, their number in *n_valid
hipError_t gwfa_launch_screen(const KArgs& A, int32_t* valid, int32_t* n_valid, hipStream_t st);

// pruning network: training and batch inference (gwfa_mlp.hip)
struct Scale8 {
    float s[8];
};
int64_t gwfa_mlp_scratch_floats(int64_t samples);
hipError_t gwfa_launch_mlp_grad(const float* feat, int64_t stride, const Scale8& scale, const uint8_t* label,
                                int64_t n, float pos_weight, const uint16_t* w, float* scr, int64_t scr_samples,
                                float* grad, float* loss, hipStream_t st);
hipError_t gwfa_launch_mlp_adam(float* master, float* m1, float* m2, const float* grad, uint16_t* wb, float lr,
                                float beta1, float beta2, float eps, float bc1, float bc2, hipStream_t st);
hipError_t gwfa_launch_mlp_cast(const float* src, uint16_t* dst, int64_t n, hipStream_t st);
hipError_t gwfa_launch_mlp_logits(const float* feat, int64_t stride, const Scale8& scale, int64_t n,
                                  const uint16_t* w, float* out, hipStream_t st);

// base-level alignment along the traced walks (gwfa_cigar.hip)
struct CigArgs {
    const unsigned long long* seg;   // packed labels
    const int64_t* seg_off;
    const unsigned long long* rd;    // packed queries
    const int64_t* rd_off;
    int32_t n_reads;
    const gwfa_result* res;
    const int32_t* path_buf;
    uint32_t* cigar;
    int64_t cigar_cap;
    unsigned long long* cigar_cursor;
    int64_t* cigar_off;
    int32_t* cigar_len;
    int32_t* queue;
    char* arena;                     // one region per workgroup
    int64_t arena_stride, o_pref, o_wf, o_ops;
    int32_t max_d, max_q, max_t;     // capacities of the regions
};
hipError_t gwfa_launch_cigar(const CigArgs& A, int groups, hipStream_t st);
