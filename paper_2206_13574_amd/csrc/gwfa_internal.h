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
    int32_t n_vtx;
    // queries (device)
    const unsigned long long* rd;    // packed queries
    const int64_t* rd_off;           // n_reads+1 base offsets
    const int32_t* v_start;
    const int32_t* order;            // work-queue order or null
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
    const uint16_t* mlp_w;           // bf16 weights (device) or null
    const float* mlp_scale;          // 8 feature scales (device) or null
    // working memory: one arena per workgroup
    char* arena;
    int64_t arena_stride;
    int32_t dir_log2_max, dir_factor, list_cap, cand_cap, sort_cap;
    int64_t o_hdr, o_dir, o_pages, o_mkey, o_tv, o_tt, o_lists, o_cand, o_sort;
};

hipError_t gwfa_launch_align(const KArgs& A, int lanes, int groups, hipStream_t st);
hipError_t gwfa_launch_pack(const uint8_t* ascii, int64_t n, unsigned long long* out, int64_t n_words,
                            int32_t* err, hipStream_t st);
hipError_t gwfa_launch_reset(int32_t* queue, unsigned long long* cursor, int32_t* retry_count, hipStream_t st);
