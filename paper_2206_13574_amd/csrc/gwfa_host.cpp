// gwfa_host.cpp -- host side of the C ABI declared in include/gwfa.h:
// contexts, graphs, working memory (per-workgroup HBM arenas in size tiers),
// validation, launches and the overflow re-run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "gwfa.h"
#include "gwfa_internal.h"

static_assert(sizeof(gwfa_result) == 64, "gwfa_result layout");

namespace {

constexpr int N_TIERS = 3;
constexpr int64_t MLP_SCR_SAMPLES = 16384;

struct Tier {
    int32_t dir_log2_max = 16;
    int32_t list_cap = 1 << 15;
    int32_t cand_cap = 1 << 16;
    int32_t sort_cap = 1 << 15;
    int32_t groups = 0;
    char* arena = nullptr;
    int64_t stride = 0;
    int64_t o_hdr = 0, o_dir = 0, o_pages = 0, o_mkey = 0, o_tv = 0, o_tt = 0, o_lists = 0, o_cand = 0, o_sort = 0;
};

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// One arena per persistent workgroup: header (generation counter), page
// directory, record pages, trace map + trace array, two wavefront lists,
// crossing candidates, sort scratch.
void layout(Tier& t) {
    const int64_t C = (int64_t)1 << t.dir_log2_max;
    t.sort_cap = 1;
    while (t.sort_cap < t.list_cap) t.sort_cap <<= 1;
    int64_t o = 0;
    t.o_hdr = o;   o = align_up(o + 256, 512);
    t.o_dir = o;   o = align_up(o + C * 8, 512);
    t.o_pages = o; o = align_up(o + C * 512, 512);
    t.o_mkey = o;  o = align_up(o + C * 8, 256);
    t.o_tv = o;    o = align_up(o + C * 4, 256);
    t.o_tt = o;    o = align_up(o + C * 4, 256);
    t.o_lists = o; o = align_up(o + (int64_t)2 * 9 * t.list_cap * 4, 256);
    t.o_cand = o;  o = align_up(o + (int64_t)4 * t.cand_cap * 4, 256);
    t.o_sort = o;  o = align_up(o + (int64_t)t.sort_cap * 12, 4096);
    t.stride = o;
}

}  // namespace

struct gwfa_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t lanes = 256;
    int32_t groups = 0;
    int32_t dir_factor = 16;
    Tier tier[N_TIERS];
    int32_t* d_queue = nullptr;
    unsigned long long* d_cursor = nullptr;
    int32_t* d_retry_count = nullptr;
    unsigned long long* d_stats = nullptr;
    int32_t* d_retry[2] = {nullptr, nullptr};
    int32_t* d_valid = nullptr;        // queries that passed the screen pass, in work-queue order
    int32_t* d_valid_n = nullptr;
    int64_t retry_cap = 0;
    int64_t rerun_total = 0;
    uint16_t* d_mlp = nullptr;
    float* d_mlp_scale = nullptr;
    bool mlp_loaded = false;
    float* d_mlp_scr = nullptr;        // training activations, MLP_SCR_SAMPLES samples
    int64_t epoch = 0;                 // bumped when working memory is freed (invalidates plans)
    char* d_cig_arena = nullptr;       // base-level alignment: per-workgroup regions
    size_t cig_bytes = 0;
    int32_t* d_cig_queue = nullptr;
    int n_cu = 256;
    char* static_base = nullptr;       // the device's static working memory (gwfa_align_batch_static_dev)
    std::string err;
};

struct gwfa_graph {
    int device = 0;                    // the graph does not depend on the context that built it
    int32_t n_vtx = 0;
    int64_t n_edge = 0;
    int64_t bases = 0;
    unsigned long long* d_seg = nullptr;
    int64_t* d_seg_off = nullptr;
    int32_t* d_out_off = nullptr;
    int32_t* d_out_dst = nullptr;
    int4* d_vinfo = nullptr;           // per vertex: first out-edge, out-degree, first two targets
    int4* d_vlab = nullptr;            // per vertex: label base (low, high 32 bits), label length, 0
};

namespace {

int dev_fail(gwfa_ctx* ctx, hipError_t e, const char* what) {
    if (ctx) {
        ctx->err = std::string(what) + ": " + hipGetErrorString(e);
    }
    return GWFA_ERR_DEVICE;
}

#define HIPCHK(ctx, call)                                              \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return dev_fail((ctx), e_, #call);       \
    } while (0)

inline bool is_acgt(uint8_t c) {
    const uint8_t u = c & 0xdf;
    return u == 'A' || u == 'C' || u == 'G' || u == 'T';
}

void free_tier(Tier& t) {
    if (t.arena) (void)hipFree(t.arena);
    t.arena = nullptr;
}

int ensure_tier(gwfa_ctx* ctx, int ti) {
    Tier& t = ctx->tier[ti];
    if (t.arena) return GWFA_OK;
    layout(t);
    size_t bytes = (size_t)t.stride * (size_t)t.groups;
    hipError_t e = hipMalloc((void**)&t.arena, bytes);
    if (e != hipSuccess) {
        t.arena = nullptr;
        ctx->err = "arena allocation of " + std::to_string(bytes) + " bytes failed";
        return GWFA_ERR_NOMEM;
    }
    // generation 0 everywhere: record words of generation 0 read as "never
    // seen" for every query (queries use generations 1, 2, ...)
    e = hipMemset(t.arena, 0, bytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();   // finished before any kernel on any stream uses it
    if (e != hipSuccess) return dev_fail(ctx, e, "arena clear");
    return GWFA_OK;
}

// Share of the device memory free at configuration time that each tier's
// arenas may take (all three can be allocated at once).
constexpr double TIER_SHARE[N_TIERS] = {0.60, 0.20, 0.05};

void set_tiers(gwfa_ctx* ctx, int32_t dir_log2_max, int32_t list_cap) {
    // default: as many persistent workgroups as can be resident at once
    int per_cu = gwfa_align_blocks_per_cu(ctx->lanes);
    if (per_cu <= 0) per_cu = 4;
    const int groups = ctx->groups > 0 ? ctx->groups : ctx->n_cu * per_cu;
    // the old arenas go first, so that the free memory the new tiers are
    // sized from includes them
    for (int i = 0; i < N_TIERS; ++i) free_tier(ctx->tier[i]);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || free_b == 0) free_b = (size_t)64 << 30;
    for (int i = 0; i < N_TIERS; ++i) {
        Tier& t = ctx->tier[i];
        t.dir_log2_max = std::min(dir_log2_max + 2 * i, 24);
        t.list_cap = (int32_t)std::min<int64_t>((int64_t)list_cap << (2 * i), (int64_t)1 << 26);
        t.cand_cap = (int32_t)std::min<int64_t>((int64_t)t.list_cap * 2, (int64_t)1 << 27);
        layout(t);
        // larger tiers keep as many workgroups as their share of memory holds:
        // queries that overflow the first tier still run at full width
        const int64_t fit = (int64_t)(TIER_SHARE[i] * (double)free_b) / t.stride;
        t.groups = (int)std::max<int64_t>(4, std::min<int64_t>(groups, fit));
    }
}

}  // namespace

extern "C" {

void gwfa_opts_default(gwfa_opts* o) {
    if (!o) return;
    o->prune = GWFA_PRUNE_NONE;
    o->a_diff = 0;
    o->keep_threshold = 0.0f;
    o->traceback = 1;
    o->max_score = -1;
    o->end_vertex = -1;
    o->mlp_gate = 0;
    o->mlp_period = 1;
    o->query_end_free = 0;
    o->walk_end_free = 0;
}

const char* gwfa_strerror(int code) {
    switch (code) {
    case GWFA_OK: return "ok";
    case GWFA_ERR_ARG: return "invalid argument";
    case GWFA_ERR_VERTEX: return "vertex id out of range";
    case GWFA_ERR_ALPHABET: return "base outside A,C,G,T";
    case GWFA_ERR_EMPTY_LABEL: return "vertex with an empty label";
    case GWFA_ERR_NOMEM: return "out of memory";
    case GWFA_ERR_DEVICE: return "HIP runtime error";
    case GWFA_ERR_PATH_CAP: return "path buffer too small";
    case GWFA_ERR_UNSUPPORTED: return "unsupported option";
    case GWFA_ERR_FORMAT: return "malformed GFA input";
    default: return "unknown error";
    }
}

const char* gwfa_last_error(const gwfa_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

int gwfa_ctx_create(int device, void* hip_stream, gwfa_ctx** out) {
    if (!out || device < 0) return GWFA_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) return GWFA_ERR_DEVICE;
    gwfa_ctx* c = new (std::nothrow) gwfa_ctx();
    if (!c) return GWFA_ERR_NOMEM;
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) { delete c; return GWFA_ERR_DEVICE; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->n_cu = prop.multiProcessorCount;
    // NULL selects the HIP null stream, which orders with every blocking
    // stream of the device (e.g. the default stream of a framework)
    c->stream = (hipStream_t)hip_stream;
    c->own_stream = false;
    bool ok = hipMalloc((void**)&c->d_queue, sizeof(int32_t)) == hipSuccess &&
              hipMalloc((void**)&c->d_cursor, sizeof(unsigned long long)) == hipSuccess &&
              hipMalloc((void**)&c->d_retry_count, sizeof(int32_t)) == hipSuccess &&
              hipMalloc((void**)&c->d_valid_n, sizeof(int32_t)) == hipSuccess &&
              hipMalloc((void**)&c->d_stats, 16 * sizeof(unsigned long long)) == hipSuccess;
    if (ok) ok = hipMemset(c->d_stats, 0, 16 * sizeof(unsigned long long)) == hipSuccess &&
                 hipDeviceSynchronize() == hipSuccess;
    if (!ok) { gwfa_ctx_destroy(c); return GWFA_ERR_NOMEM; }
    set_tiers(c, 16, 1 << 15);
    // the static working memory of this device (looked up and cleared on the
    // first context of the process); its entry point reports a failure here
    c->static_base = (char*)gwfa_static_scratch(device);
    *out = c;
    return GWFA_OK;
}

void gwfa_ctx_destroy(gwfa_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& t : c->tier) free_tier(t);
    if (c->d_queue) (void)hipFree(c->d_queue);
    if (c->d_cursor) (void)hipFree(c->d_cursor);
    if (c->d_retry_count) (void)hipFree(c->d_retry_count);
    if (c->d_stats) (void)hipFree(c->d_stats);
    for (auto p : c->d_retry) if (p) (void)hipFree(p);
    if (c->d_valid) (void)hipFree(c->d_valid);
    if (c->d_valid_n) (void)hipFree(c->d_valid_n);
    if (c->d_mlp) (void)hipFree(c->d_mlp);
    if (c->d_mlp_scale) (void)hipFree(c->d_mlp_scale);
    if (c->d_mlp_scr) (void)hipFree(c->d_mlp_scr);
    if (c->d_cig_arena) (void)hipFree(c->d_cig_arena);
    if (c->d_cig_queue) (void)hipFree(c->d_cig_queue);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int gwfa_ctx_config(gwfa_ctx* c, int32_t lanes, int32_t n_groups, int32_t dir_log2_max, int32_t list_cap,
                    int32_t dir_factor) {
    if (!c) return GWFA_ERR_ARG;
    if (lanes != 64 && lanes != 128 && lanes != 256 && lanes != 512) return GWFA_ERR_ARG;
    if (n_groups < 0 || n_groups > (1 << 20)) return GWFA_ERR_ARG;
    if (dir_log2_max < 10 || dir_log2_max > 22) return GWFA_ERR_ARG;
    if (list_cap < 1024 || list_cap > (1 << 24) || (list_cap & 1)) return GWFA_ERR_ARG;
    if (dir_factor < 1 || dir_factor > 4096 || (dir_factor & (dir_factor - 1))) return GWFA_ERR_ARG;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    c->lanes = lanes;
    c->groups = n_groups;
    c->dir_factor = dir_factor;
    set_tiers(c, dir_log2_max, list_cap);
    c->epoch++;
    return GWFA_OK;
}

int64_t gwfa_packed_words(int64_t n_bases) { return n_bases < 0 ? 0 : (n_bases + 31) / 32 + 2; }

int gwfa_graph_create(gwfa_ctx* ctx, int32_t n_vtx, const uint8_t* seq, const int64_t* seq_off, int64_t n_edge,
                      const int32_t* edge_src, const int32_t* edge_dst, gwfa_graph** out) {
    if (!ctx || !out || n_vtx <= 0 || !seq_off || n_edge < 0) return GWFA_ERR_ARG;
    if (n_edge > 0 && (!edge_src || !edge_dst)) return GWFA_ERR_ARG;
    *out = nullptr;
    if (seq_off[0] != 0) return GWFA_ERR_ARG;
    for (int32_t v = 0; v < n_vtx; ++v) {
        if (seq_off[v + 1] < seq_off[v]) return GWFA_ERR_ARG;
        if (seq_off[v + 1] == seq_off[v]) return GWFA_ERR_EMPTY_LABEL;
    }
    const int64_t bases = seq_off[n_vtx];
    if (bases > 0 && !seq) return GWFA_ERR_ARG;
    if (bases >= ((int64_t)1 << 40)) return GWFA_ERR_ARG;
    for (int64_t i = 0; i < bases; ++i)
        if (!is_acgt(seq[i])) return GWFA_ERR_ALPHABET;
    for (int32_t v = 0; v < n_vtx; ++v)
        if (seq_off[v + 1] - seq_off[v] > (int64_t)1 << 30) return GWFA_ERR_ARG;
    for (int64_t e = 0; e < n_edge; ++e)
        if (edge_src[e] < 0 || edge_src[e] >= n_vtx || edge_dst[e] < 0 || edge_dst[e] >= n_vtx) return GWFA_ERR_VERTEX;
    if (n_edge > INT32_MAX) return GWFA_ERR_ARG;

    // out-edge CSR (edges of a vertex keep their input order)
    std::vector<int32_t> off(n_vtx + 1, 0), dst((size_t)std::max<int64_t>(n_edge, 1));
    for (int64_t e = 0; e < n_edge; ++e) off[edge_src[e] + 1]++;
    for (int32_t v = 0; v < n_vtx; ++v) off[v + 1] += off[v];
    {
        std::vector<int32_t> fill(off.begin(), off.end() - 1);
        for (int64_t e = 0; e < n_edge; ++e) dst[fill[edge_src[e]]++] = edge_dst[e];
    }
    // per-vertex out-edge record: one 16-byte load gives a vertex's edge range
    // and its first two targets (most vertices of a sequence graph have at
    // most two successors)
    std::vector<int4> vinfo((size_t)n_vtx);
    for (int32_t v = 0; v < n_vtx; ++v) {
        const int32_t b = off[v], d = off[v + 1] - off[v];
        vinfo[v] = make_int4(b, d, d > 0 ? dst[b] : -1, d > 1 ? dst[b + 1] : -1);
    }
    // per-vertex label record: one 16-byte load gives the base and length
    // of a vertex's label in the packed store
    std::vector<int4> vlab((size_t)n_vtx);
    for (int32_t v = 0; v < n_vtx; ++v) {
        const uint64_t b = (uint64_t)seq_off[v];
        vlab[v] = make_int4((int32_t)(uint32_t)b, (int32_t)(uint32_t)(b >> 32), (int32_t)(seq_off[v + 1] - seq_off[v]), 0);
    }
    gwfa_graph* g = new (std::nothrow) gwfa_graph();
    if (!g) return GWFA_ERR_NOMEM;
    g->device = ctx->device; g->n_vtx = n_vtx; g->n_edge = n_edge; g->bases = bases;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int64_t words = gwfa_packed_words(bases);
    uint8_t* d_ascii = nullptr;
    int32_t* d_err = nullptr;
    bool ok = hipMalloc((void**)&g->d_seg, words * 8) == hipSuccess &&
              hipMalloc((void**)&g->d_seg_off, (size_t)(n_vtx + 1) * 8) == hipSuccess &&
              hipMalloc((void**)&g->d_out_off, (size_t)(n_vtx + 1) * 4) == hipSuccess &&
              hipMalloc((void**)&g->d_out_dst, dst.size() * 4) == hipSuccess &&
              hipMalloc((void**)&g->d_vinfo, (size_t)n_vtx * sizeof(int4)) == hipSuccess &&
              hipMalloc((void**)&g->d_vlab, (size_t)n_vtx * sizeof(int4)) == hipSuccess &&
              hipMalloc((void**)&d_ascii, (size_t)std::max<int64_t>(bases, 1)) == hipSuccess &&
              hipMalloc((void**)&d_err, 4) == hipSuccess;
    if (!ok) {
        if (d_ascii) (void)hipFree(d_ascii);
        if (d_err) (void)hipFree(d_err);
        gwfa_graph_destroy(g);
        return GWFA_ERR_NOMEM;
    }
    hipStream_t st = ctx->stream;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(d_ascii, seq, (size_t)bases, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(d_err, 0, 4, st);
    if (e == hipSuccess) e = gwfa_launch_pack(d_ascii, bases, g->d_seg, words, d_err, st);
    if (e == hipSuccess) e = hipMemcpyAsync(g->d_seg_off, seq_off, (size_t)(n_vtx + 1) * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(g->d_out_off, off.data(), (size_t)(n_vtx + 1) * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(g->d_out_dst, dst.data(), dst.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_vinfo, vinfo.data(), vinfo.size() * sizeof(int4), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_vlab, vlab.data(), vlab.size() * sizeof(int4), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_ascii);
    (void)hipFree(d_err);
    if (e != hipSuccess) {
        gwfa_graph_destroy(g);
        return dev_fail(ctx, e, "graph upload");
    }
    *out = g;
    return GWFA_OK;
}

void gwfa_graph_destroy(gwfa_graph* g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    if (g->d_seg) (void)hipFree(g->d_seg);
    if (g->d_seg_off) (void)hipFree(g->d_seg_off);
    if (g->d_out_off) (void)hipFree(g->d_out_off);
    if (g->d_out_dst) (void)hipFree(g->d_out_dst);
    if (g->d_vinfo) (void)hipFree(g->d_vinfo);
    if (g->d_vlab) (void)hipFree(g->d_vlab);
    delete g;
}

int gwfa_pack_dev(gwfa_ctx* ctx, const uint8_t* d_ascii, int64_t n_bases, uint64_t* d_packed, int32_t* d_err,
                  void* hip_stream) {
    if (!ctx || n_bases < 0 || !d_packed || (n_bases > 0 && !d_ascii)) return GWFA_ERR_ARG;
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, gwfa_launch_pack(d_ascii, n_bases, (unsigned long long*)d_packed, gwfa_packed_words(n_bases), d_err, st));
    return GWFA_OK;
}

static int check_opts(const gwfa_ctx* ctx, const gwfa_opts* o) {
    if (!o) return GWFA_ERR_ARG;
    if (o->end_vertex < -1) return GWFA_ERR_ARG;
    if (o->prune < 0 || o->prune > 2) return GWFA_ERR_ARG;
    if (o->prune == GWFA_PRUNE_HEURISTIC && o->a_diff < 1) return GWFA_ERR_ARG;
    if (o->prune == GWFA_PRUNE_LEARNED) {
        if (!ctx->mlp_loaded) return GWFA_ERR_UNSUPPORTED;
        if (o->mlp_period < 1 || o->mlp_gate < 0) return GWFA_ERR_ARG;
    }
    if (o->max_score < -1) return GWFA_ERR_ARG;
    if (o->query_end_free < 0) return GWFA_ERR_ARG;
    if (o->walk_end_free != 0 && o->walk_end_free != 1) return GWFA_ERR_ARG;
    if (o->traceback != 0 && o->traceback != 1) return GWFA_ERR_ARG;
    return GWFA_OK;
}

// Launch arguments common to every tier of one batch.
static int fill_args(gwfa_ctx* ctx, const gwfa_graph* g, int32_t n_reads, const uint64_t* d_packed,
                     const int64_t* d_read_off, const int32_t* d_v_start, const int32_t* d_v_end,
                     const gwfa_opts* opts, gwfa_result* d_res, int32_t* d_path_buf, int64_t path_cap,
                     int64_t* d_path_used, float* d_dump, int64_t dump_cap, int64_t* d_dump_count, KArgs& A) {
    if (!ctx || !g || n_reads < 0 || path_cap < 0) return GWFA_ERR_ARG;
    if (g->device != ctx->device) return GWFA_ERR_ARG;
    int rc = check_opts(ctx, opts);
    if (rc) return rc;
    if (opts->end_vertex >= g->n_vtx) return GWFA_ERR_VERTEX;
    if (d_v_end && opts->end_vertex >= 0) return GWFA_ERR_ARG;
    if (n_reads > 0 && (!d_packed || !d_read_off || !d_v_start || !d_res)) return GWFA_ERR_ARG;
    memset(&A, 0, sizeof(A));
    A.seg = g->d_seg; A.seg_off = g->d_seg_off; A.out_off = g->d_out_off; A.out_dst = g->d_out_dst;
    A.vinfo = g->d_vinfo; A.vlab = g->d_vlab; A.n_vtx = g->n_vtx;
    A.rd = (const unsigned long long*)d_packed; A.rd_off = d_read_off; A.v_start = d_v_start;
    A.v_end = d_v_end; A.end_vertex = opts->end_vertex;
    A.res = d_res; A.path_buf = d_path_buf; A.path_cap = d_path_buf ? path_cap : 0;
    A.path_cursor = d_path_used ? (unsigned long long*)d_path_used : ctx->d_cursor;
    A.queue = ctx->d_queue; A.stats = ctx->d_stats;
    A.retry_count = ctx->d_retry_count;
    A.prune = opts->prune; A.a_diff = opts->a_diff; A.traceback = opts->traceback; A.max_score = opts->max_score;
    A.keep_threshold = opts->keep_threshold; A.mlp_gate = opts->mlp_gate; A.mlp_period = opts->mlp_period;
    A.end_free = opts->query_end_free;
    A.walk_free = opts->walk_end_free;
    A.mlp_w = ctx->d_mlp; A.mlp_scale = ctx->d_mlp_scale;
    A.dir_factor = ctx->dir_factor;
    A.dump = d_dump; A.dump_cap = d_dump ? dump_cap : 0; A.dump_count = (unsigned long long*)d_dump_count;
    return GWFA_OK;
}

// The context's per-query lists (screened queries, re-run lists) for a batch
// of n_reads queries.
static int ensure_lists(gwfa_ctx* ctx, int32_t n_reads) {
    if (ctx->retry_cap >= n_reads) return GWFA_OK;
    for (auto& p : ctx->d_retry) { if (p) (void)hipFree(p); p = nullptr; }
    if (ctx->d_valid) (void)hipFree(ctx->d_valid);
    ctx->d_valid = nullptr;
    ctx->retry_cap = 0;
    ctx->epoch++;   // captured plans hold the old lists
    for (auto& p : ctx->d_retry)
        if (hipMalloc((void**)&p, (size_t)n_reads * 4) != hipSuccess) { p = nullptr; return GWFA_ERR_NOMEM; }
    if (hipMalloc((void**)&ctx->d_valid, (size_t)n_reads * 4) != hipSuccess) {
        ctx->d_valid = nullptr;
        return GWFA_ERR_NOMEM;
    }
    ctx->retry_cap = n_reads;
    return GWFA_OK;
}

// Working memory of tier ti into A; returns the workgroups to launch.
static int set_tier(gwfa_ctx* ctx, KArgs& A, int ti, const int32_t* order, int32_t n, const int32_t* n_valid,
                    int* groups) {
    int rc = ensure_tier(ctx, ti);
    if (rc) return rc;
    const Tier& t = ctx->tier[ti];
    A.order = order; A.n_reads = n; A.n_valid = n_valid; A.tier = ti;
    A.retry = (ti + 1 < N_TIERS) ? ctx->d_retry[ti & 1] : nullptr;
    A.arena = t.arena; A.arena_stride = t.stride;
    A.dir_log2_max = t.dir_log2_max; A.list_cap = t.list_cap; A.cand_cap = t.cand_cap; A.sort_cap = t.sort_cap;
    A.o_hdr = t.o_hdr; A.o_dir = t.o_dir; A.o_pages = t.o_pages; A.o_mkey = t.o_mkey;
    A.o_tv = t.o_tv; A.o_tt = t.o_tt; A.o_lists = t.o_lists; A.o_cand = t.o_cand; A.o_sort = t.o_sort;
    *groups = (int)std::min<int64_t>(t.groups, n);
    return GWFA_OK;
}

// Tiers ti0, ti0+1, ...: after each launch the queries that overflowed
// their working memory (if any) are re-run on the next, larger tier.  When
// `launched` the launch of tier ti0 has already been issued.  The first
// tier takes the queries the screen pass listed (ctx->d_valid, their number
// on the device); a re-run takes the retry list of the tier before.
static int run_tiers(gwfa_ctx* ctx, KArgs& A, int ti0, int32_t n, bool launched, hipStream_t st) {
    const int32_t* order = ctx->d_valid;
    const int32_t* n_valid = ctx->d_valid_n;
    for (int ti = ti0; ti < N_TIERS; ++ti) {
        if (!(launched && ti == ti0)) {
            int groups = 0;
            int rc = set_tier(ctx, A, ti, order, n, n_valid, &groups);
            if (rc) return rc;
            HIPCHK(ctx, gwfa_launch_align(A, ctx->lanes, groups, st));
        }
        if (ti + 1 == N_TIERS) break;
        int32_t h_retry = 0;
        HIPCHK(ctx, hipMemcpyAsync(&h_retry, ctx->d_retry_count, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        if (h_retry <= 0) break;
        ctx->rerun_total += h_retry;
        order = ctx->d_retry[ti & 1];
        n = h_retry;
        n_valid = nullptr;
        // reset the queue and the retry counter, keep the path cursor and the dump counter
        HIPCHK(ctx, gwfa_launch_reset(ctx->d_queue, nullptr, ctx->d_retry_count, nullptr, st));
    }
    return GWFA_OK;
}

static int align_dev(gwfa_ctx* ctx, const gwfa_graph* g, int32_t n_reads, const uint64_t* d_packed,
                     const int64_t* d_read_off, const int32_t* d_v_start, const int32_t* d_v_end,
                     const int32_t* d_order, const gwfa_opts* opts, gwfa_result* d_res, int32_t* d_path_buf,
                     int64_t path_cap, int64_t* d_path_used, float* d_dump, int64_t dump_cap,
                     int64_t* d_dump_count, void* hip_stream, const int32_t* d_start_off = nullptr,
                     const int32_t* d_start_hi = nullptr) {
    if (!ctx) return GWFA_ERR_ARG;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    KArgs A;
    int rc = fill_args(ctx, g, n_reads, d_packed, d_read_off, d_v_start, d_v_end, opts, d_res, d_path_buf,
                       path_cap, d_path_used, d_dump, dump_cap, d_dump_count, A);
    if (!rc) rc = ensure_lists(ctx, n_reads);
    if (rc || n_reads == 0) return rc;
    A.v_off = d_start_off;
    A.v_off_hi = d_start_hi;
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIPCHK(ctx, gwfa_launch_reset(ctx->d_queue, A.path_cursor, ctx->d_retry_count, A.dump_count, st));
    A.order = d_order;
    A.n_reads = n_reads;
    HIPCHK(ctx, gwfa_launch_screen(A, ctx->d_valid, ctx->d_valid_n, st));
    return run_tiers(ctx, A, 0, n_reads, false, st);
}

int gwfa_align_batch_dev(gwfa_ctx* ctx, const gwfa_graph* g, int32_t n_reads, const uint64_t* d_packed,
                         const int64_t* d_read_off, const int32_t* d_v_start, const int32_t* d_order,
                         const gwfa_opts* opts, gwfa_result* d_res, int32_t* d_path_buf, int64_t path_cap,
                         int64_t* d_path_used, void* hip_stream) {
    return align_dev(ctx, g, n_reads, d_packed, d_read_off, d_v_start, nullptr, d_order, opts, d_res, d_path_buf,
                     path_cap, d_path_used, nullptr, 0, nullptr, hip_stream);
}

int gwfa_align_global_dev(gwfa_ctx* ctx, const gwfa_graph* g, int32_t n_reads, const uint64_t* d_packed,
                          const int64_t* d_read_off, const int32_t* d_v_start, const int32_t* d_v_end,
                          const int32_t* d_order, const gwfa_opts* opts, gwfa_result* d_res, int32_t* d_path_buf,
                          int64_t path_cap, int64_t* d_path_used, void* hip_stream) {
    if (n_reads > 0 && !d_v_end) return GWFA_ERR_ARG;
    return align_dev(ctx, g, n_reads, d_packed, d_read_off, d_v_start, d_v_end, d_order, opts, d_res, d_path_buf,
                     path_cap, d_path_used, nullptr, 0, nullptr, hip_stream);
}

int gwfa_align_at_dev(gwfa_ctx* ctx, const gwfa_graph* g, int32_t n_reads, const uint64_t* d_packed,
                      const int64_t* d_read_off, const int32_t* d_v_start, const int32_t* d_start_off,
                      const int32_t* d_start_hi, const int32_t* d_v_end, const int32_t* d_order,
                      const gwfa_opts* opts, gwfa_result* d_res, int32_t* d_path_buf, int64_t path_cap,
                      int64_t* d_path_used, void* hip_stream) {
    if (n_reads > 0 && d_start_hi && !d_start_off) return GWFA_ERR_ARG;
    return align_dev(ctx, g, n_reads, d_packed, d_read_off, d_v_start, d_v_end, d_order, opts, d_res, d_path_buf,
                     path_cap, d_path_used, nullptr, 0, nullptr, hip_stream, d_start_off, d_start_hi);
}

int gwfa_align_dump_dev(gwfa_ctx* ctx, const gwfa_graph* g, int32_t n_reads, const uint64_t* d_packed,
                        const int64_t* d_read_off, const int32_t* d_v_start, const int32_t* d_order,
                        const gwfa_opts* opts, gwfa_result* d_res, int32_t* d_path_buf, int64_t path_cap,
                        int64_t* d_path_used, float* d_dump, int64_t dump_cap, int64_t* d_dump_count,
                        void* hip_stream) {
    if (!d_dump || dump_cap < 0 || !d_dump_count) return GWFA_ERR_ARG;
    return align_dev(ctx, g, n_reads, d_packed, d_read_off, d_v_start, nullptr, d_order, opts, d_res, d_path_buf,
                     path_cap, d_path_used, d_dump, dump_cap, d_dump_count, hip_stream);
}

int gwfa_align_batch_static_dev(gwfa_ctx* ctx, const gwfa_graph* g, int32_t n_reads, const uint64_t* d_packed,
                                const int64_t* d_read_off, const int32_t* d_v_start, const int32_t* d_order,
                                const gwfa_opts* opts, gwfa_result* d_res, int32_t* d_path_buf, int64_t path_cap,
                                int64_t* d_path_used, void* hip_stream) {
    if (!ctx) return GWFA_ERR_ARG;
    if (n_reads > STATIC_MAX_READS) {
        ctx->err = "gwfa_align_batch_static_dev takes at most " + std::to_string(STATIC_MAX_READS) +
                   " queries per call, got " + std::to_string(n_reads);
        return GWFA_ERR_ARG;
    }
    if (!ctx->static_base) {
        ctx->err = "the static working memory of this device could not be set up";
        return GWFA_ERR_DEVICE;
    }
    HIPCHK(ctx, hipSetDevice(ctx->device));
    KArgs A;
    int rc = fill_args(ctx, g, n_reads, d_packed, d_read_off, d_v_start, nullptr, opts, d_res, d_path_buf,
                       path_cap, d_path_used, nullptr, 0, nullptr, A);
    if (rc || n_reads == 0) return rc;
    // layout of the static array: header, screened list, one tier of arenas
    char* base = ctx->static_base;
    int32_t* queue = reinterpret_cast<int32_t*>(base);
    int32_t* retry_count = queue + 1;
    int32_t* n_valid = queue + 2;
    unsigned long long* cursor = reinterpret_cast<unsigned long long*>(base + 64);
    int32_t* valid = reinterpret_cast<int32_t*>(base + STATIC_HDR);
    const int64_t o_arenas = align_up(STATIC_HDR + (int64_t)STATIC_MAX_READS * 4, 4096);
    Tier t;
    t.dir_log2_max = STATIC_DIR_LOG2;
    t.list_cap = STATIC_LIST_CAP;
    t.cand_cap = 2 * STATIC_LIST_CAP;
    layout(t);
    int per_cu = gwfa_align_blocks_per_cu(ctx->lanes);
    if (per_cu <= 0) per_cu = 4;
    const int64_t fit = (STATIC_BYTES - o_arenas) / t.stride;
    const int groups = (int)std::min<int64_t>(std::min<int64_t>(fit, (int64_t)ctx->n_cu * per_cu), n_reads);
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    A.queue = queue;
    A.retry_count = retry_count;
    A.retry = nullptr;   // one tier: a query that overflows it keeps GWFA_ST_ARENA
    if (!d_path_used) A.path_cursor = cursor;
    HIPCHK(ctx, gwfa_launch_reset(queue, A.path_cursor, retry_count, nullptr, st));
    A.order = d_order;
    A.n_reads = n_reads;
    HIPCHK(ctx, gwfa_launch_screen(A, valid, n_valid, st));
    A.order = valid; A.n_valid = n_valid; A.tier = 0;
    A.arena = base + o_arenas; A.arena_stride = t.stride;
    A.dir_log2_max = t.dir_log2_max; A.list_cap = t.list_cap; A.cand_cap = t.cand_cap; A.sort_cap = t.sort_cap;
    A.o_hdr = t.o_hdr; A.o_dir = t.o_dir; A.o_pages = t.o_pages; A.o_mkey = t.o_mkey;
    A.o_tv = t.o_tv; A.o_tt = t.o_tt; A.o_lists = t.o_lists; A.o_cand = t.o_cand; A.o_sort = t.o_sort;
    HIPCHK(ctx, gwfa_launch_align(A, ctx->lanes, groups, st));
    return GWFA_OK;
}

struct gwfa_plan {
    gwfa_ctx* ctx = nullptr;
    int device = 0;
    int64_t epoch = 0;
    KArgs A;
    const int32_t* order = nullptr;
    int32_t n_reads = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

void gwfa_plan_destroy(gwfa_plan* p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    delete p;
}

int gwfa_plan_create(gwfa_ctx* ctx, const gwfa_graph* g, int32_t n_reads, const uint64_t* d_packed,
                     const int64_t* d_read_off, const int32_t* d_v_start, const int32_t* d_order,
                     const gwfa_opts* opts, gwfa_result* d_res, int32_t* d_path_buf, int64_t path_cap,
                     int64_t* d_path_used, gwfa_plan** out) {
    if (!ctx || !out || n_reads < 1) return GWFA_ERR_ARG;
    *out = nullptr;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    gwfa_plan* p = new (std::nothrow) gwfa_plan();
    if (!p) return GWFA_ERR_NOMEM;
    p->ctx = ctx;
    p->device = ctx->device;
    p->order = d_order;
    p->n_reads = n_reads;
    int rc = fill_args(ctx, g, n_reads, d_packed, d_read_off, d_v_start, nullptr, opts, d_res, d_path_buf,
                       path_cap, d_path_used, nullptr, 0, nullptr, p->A);
    if (!rc) rc = ensure_lists(ctx, n_reads);
    int groups = 0;
    KArgs S0 = p->A;   // the screen pass reads the caller's order
    S0.order = d_order;
    S0.n_reads = n_reads;
    if (!rc) rc = set_tier(ctx, p->A, 0, ctx->d_valid, n_reads, ctx->d_valid_n, &groups);   // allocates before the capture
    if (rc) { gwfa_plan_destroy(p); return rc; }
    p->epoch = ctx->epoch;   // after any reallocation of the context's lists
    hipError_t e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        // kernels only (no memset nodes): reset of the queue and counters, the
        // screen pass, then the first tier
        hipError_t e1 = gwfa_launch_reset(ctx->d_queue, p->A.path_cursor, ctx->d_retry_count, nullptr, p->cap);
        if (e1 == hipSuccess) e1 = gwfa_launch_screen(S0, ctx->d_valid, ctx->d_valid_n, p->cap);
        if (e1 == hipSuccess) e1 = gwfa_launch_align(p->A, ctx->lanes, groups, p->cap);
        e = hipStreamEndCapture(p->cap, &p->graph);
        if (e1 != hipSuccess) e = e1;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        rc = dev_fail(ctx, e, "plan capture");
        gwfa_plan_destroy(p);
        return rc;
    }
    *out = p;
    return GWFA_OK;
}

int gwfa_plan_launch(gwfa_plan* p, void* hip_stream) {
    if (!p) return GWFA_ERR_ARG;
    gwfa_ctx* ctx = p->ctx;
    if (p->epoch != ctx->epoch) return GWFA_ERR_ARG;
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, hipGraphLaunch(p->exec, st));
    return GWFA_OK;
}

int gwfa_plan_finish(gwfa_plan* p, void* hip_stream) {
    if (!p) return GWFA_ERR_ARG;
    gwfa_ctx* ctx = p->ctx;
    if (p->epoch != ctx->epoch) return GWFA_ERR_ARG;
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    KArgs A = p->A;
    return run_tiers(ctx, A, 0, p->n_reads, true, st);
}

int gwfa_align_batch(gwfa_ctx* ctx, const gwfa_graph* g, int32_t n_reads, const uint8_t* reads,
                     const int64_t* read_off, const int32_t* v_start, const gwfa_opts* opts, gwfa_result* res,
                     int32_t* path_buf, int64_t path_cap, int64_t* path_needed) {
    if (!ctx || !g || n_reads < 0 || path_cap < 0) return GWFA_ERR_ARG;
    int rc = check_opts(ctx, opts);
    if (rc) return rc;
    if (path_needed) *path_needed = 0;
    if (opts->end_vertex >= g->n_vtx) return GWFA_ERR_VERTEX;
    if (n_reads == 0) return GWFA_OK;
    if (!read_off || !v_start || !res) return GWFA_ERR_ARG;
    if (read_off[0] != 0) return GWFA_ERR_ARG;
    for (int32_t r = 0; r < n_reads; ++r) {
        if (read_off[r + 1] < read_off[r]) return GWFA_ERR_ARG;
        if (read_off[r + 1] - read_off[r] > ((int64_t)1 << 30)) return GWFA_ERR_ARG;
        if (v_start[r] < 0 || v_start[r] >= g->n_vtx) return GWFA_ERR_VERTEX;
    }
    const int64_t bases = read_off[n_reads];
    if (bases > 0 && !reads) return GWFA_ERR_ARG;
    for (int64_t i = 0; i < bases; ++i)
        if (!is_acgt(reads[i])) return GWFA_ERR_ALPHABET;
    // longest queries first
    std::vector<int32_t> order(n_reads);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return read_off[a + 1] - read_off[a] > read_off[b + 1] - read_off[b];
    });
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int64_t words = gwfa_packed_words(bases);
    uint8_t* d_ascii = nullptr;
    unsigned long long* d_packed = nullptr;
    int64_t* d_off = nullptr;
    int32_t *d_vs = nullptr, *d_order = nullptr, *d_err = nullptr, *d_path = nullptr;
    gwfa_result* d_res = nullptr;
    int64_t* d_used = nullptr;
    const bool want_path = opts->traceback && path_buf && path_cap > 0;
    bool ok = hipMalloc((void**)&d_ascii, (size_t)std::max<int64_t>(bases, 1)) == hipSuccess &&
              hipMalloc((void**)&d_packed, (size_t)words * 8) == hipSuccess &&
              hipMalloc((void**)&d_off, (size_t)(n_reads + 1) * 8) == hipSuccess &&
              hipMalloc((void**)&d_vs, (size_t)n_reads * 4) == hipSuccess &&
              hipMalloc((void**)&d_order, (size_t)n_reads * 4) == hipSuccess &&
              hipMalloc((void**)&d_err, 4) == hipSuccess &&
              hipMalloc((void**)&d_res, (size_t)n_reads * sizeof(gwfa_result)) == hipSuccess &&
              hipMalloc((void**)&d_used, 8) == hipSuccess &&
              (!want_path || hipMalloc((void**)&d_path, (size_t)path_cap * 4) == hipSuccess);
    int out_rc = ok ? GWFA_OK : GWFA_ERR_NOMEM;
    hipError_t e = hipSuccess;
    if (ok) {
        if (e == hipSuccess) e = hipMemcpyAsync(d_ascii, reads, (size_t)bases, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(d_off, read_off, (size_t)(n_reads + 1) * 8, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(d_vs, v_start, (size_t)n_reads * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(d_order, order.data(), (size_t)n_reads * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemsetAsync(d_err, 0, 4, st);
        if (e == hipSuccess) e = gwfa_launch_pack(d_ascii, bases, d_packed, words, d_err, st);
        if (e != hipSuccess) out_rc = dev_fail(ctx, e, "query upload");
    }
    if (out_rc == GWFA_OK)
        out_rc = gwfa_align_batch_dev(ctx, g, n_reads, (const uint64_t*)d_packed, d_off, d_vs, d_order, opts, d_res,
                                      want_path ? d_path : nullptr, want_path ? path_cap : 0, d_used, st);
    if (out_rc == GWFA_OK) {
        int64_t used = 0;
        e = hipMemcpyAsync(res, d_res, (size_t)n_reads * sizeof(gwfa_result), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&used, d_used, 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess && want_path && used > 0)
            e = hipMemcpy(path_buf, d_path, (size_t)std::min(used, path_cap) * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) out_rc = dev_fail(ctx, e, "result download");
        if (out_rc == GWFA_OK) {
            if (path_needed) *path_needed = opts->traceback ? used : 0;
            if (opts->traceback && used > (want_path ? path_cap : 0)) out_rc = GWFA_ERR_PATH_CAP;
        }
    }
    if (d_ascii) (void)hipFree(d_ascii);
    if (d_packed) (void)hipFree(d_packed);
    if (d_off) (void)hipFree(d_off);
    if (d_vs) (void)hipFree(d_vs);
    if (d_order) (void)hipFree(d_order);
    if (d_err) (void)hipFree(d_err);
    if (d_res) (void)hipFree(d_res);
    if (d_used) (void)hipFree(d_used);
    if (d_path) (void)hipFree(d_path);
    return out_rc;
}

int gwfa_align(gwfa_ctx* ctx, const gwfa_graph* g, const uint8_t* q, int32_t qlen, int32_t v_start,
               const gwfa_opts* opts, gwfa_result* res, int32_t* path_buf, int64_t path_cap) {
    if (qlen < 0 || !res) return GWFA_ERR_ARG;
    const int64_t off[2] = {0, qlen};
    return gwfa_align_batch(ctx, g, 1, q, off, &v_start, opts, res, path_buf, path_cap, nullptr);
}

int gwfa_mlp_load(gwfa_ctx* ctx, const uint16_t* w, int64_t n, const float* scale) {
    if (!ctx || !w || !scale || n != 4801) return GWFA_ERR_ARG;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (!ctx->d_mlp) HIPCHK(ctx, hipMalloc((void**)&ctx->d_mlp, 4808 * 2));
    if (!ctx->d_mlp_scale) HIPCHK(ctx, hipMalloc((void**)&ctx->d_mlp_scale, 8 * 4));
    HIPCHK(ctx, hipMemcpy(ctx->d_mlp, w, (size_t)n * 2, hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemcpy(ctx->d_mlp_scale, scale, 8 * 4, hipMemcpyHostToDevice));
    ctx->mlp_loaded = true;
    return GWFA_OK;
}

int gwfa_cigar_dev(gwfa_ctx* ctx, const gwfa_graph* g, int32_t n_reads, const uint64_t* d_packed,
                   const int64_t* d_read_off, const gwfa_result* d_res, const int32_t* d_path_buf, uint32_t* d_cigar,
                   int64_t cigar_cap, int64_t* d_cigar_off, int32_t* d_cigar_len, int64_t* d_cigar_used,
                   void* hip_stream) {
    if (!ctx || !g || n_reads < 0 || cigar_cap < 0 || g->device != ctx->device) return GWFA_ERR_ARG;
    if (n_reads == 0) return GWFA_OK;
    if (!d_packed || !d_read_off || !d_res || !d_path_buf || !d_cigar_off || !d_cigar_len || !d_cigar_used ||
        (cigar_cap > 0 && !d_cigar))
        return GWFA_ERR_ARG;
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    // sizes of the per-workgroup regions from the results (one synchronisation)
    std::vector<gwfa_result> res((size_t)n_reads);
    std::vector<int64_t> off((size_t)n_reads + 1);
    HIPCHK(ctx, hipMemcpyAsync(res.data(), d_res, res.size() * sizeof(gwfa_result), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipMemcpyAsync(off.data(), d_read_off, off.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    int64_t max_d = 0, max_q = 0, max_path = 1, n_ok = 0;
    for (int32_t r = 0; r < n_reads; ++r) {
        const gwfa_result& x = res[r];
        if (x.status != GWFA_ST_OK || x.path_off < 0 || x.path_len <= 0) continue;
        ++n_ok;
        max_d = std::max<int64_t>(max_d, x.dist);
        max_q = std::max<int64_t>(max_q, off[r + 1] - off[r]);
        max_path = std::max<int64_t>(max_path, x.path_len);
    }
    // the walk's string is at most |q| + d long (its edit distance to q is <= d)
    const int64_t max_t = max_q + max_d;
    if (max_t >= ((int64_t)1 << 31) || max_d > 46000) return GWFA_ERR_UNSUPPORTED;
    CigArgs A;
    memset(&A, 0, sizeof(A));
    A.o_pref = align_up((max_t / 32 + 3) * 8, 256);
    A.o_wf = A.o_pref + align_up((max_path + 2) * 8, 256);
    A.o_ops = A.o_wf + align_up((max_d + 1) * (max_d + 1) * 4, 256);
    A.arena_stride = A.o_ops + align_up((2 * max_d + 4) * 4, 4096);
    // as many workgroups as fit in a 16 GiB region, at most two per compute unit
    int64_t groups = std::min<int64_t>(std::max<int64_t>(n_ok, 1), (int64_t)ctx->n_cu * 2);
    groups = std::max<int64_t>(1, std::min<int64_t>(groups, ((int64_t)16 << 30) / A.arena_stride));
    const size_t need = (size_t)(A.arena_stride * groups);
    if (need > ctx->cig_bytes) {
        if (ctx->d_cig_arena) (void)hipFree(ctx->d_cig_arena);
        ctx->d_cig_arena = nullptr;
        ctx->cig_bytes = 0;
        if (hipMalloc((void**)&ctx->d_cig_arena, need) != hipSuccess) {
            ctx->d_cig_arena = nullptr;
            return GWFA_ERR_NOMEM;
        }
        ctx->cig_bytes = need;
    }
    if (!ctx->d_cig_queue && hipMalloc((void**)&ctx->d_cig_queue, 4) != hipSuccess) {
        ctx->d_cig_queue = nullptr;
        return GWFA_ERR_NOMEM;
    }
    A.seg = g->d_seg; A.seg_off = g->d_seg_off;
    A.rd = (const unsigned long long*)d_packed; A.rd_off = d_read_off; A.n_reads = n_reads;
    A.res = d_res; A.path_buf = d_path_buf;
    A.cigar = d_cigar; A.cigar_cap = d_cigar ? cigar_cap : 0;
    A.cigar_cursor = (unsigned long long*)d_cigar_used;
    A.cigar_off = d_cigar_off; A.cigar_len = d_cigar_len;
    A.queue = ctx->d_cig_queue;
    A.arena = ctx->d_cig_arena;
    A.max_d = (int32_t)max_d; A.max_q = (int32_t)max_q; A.max_t = (int32_t)max_t;
    HIPCHK(ctx, gwfa_launch_cigar(A, (int)groups, st));
    return GWFA_OK;
}

static bool get_scale(const float* h, Scale8& s) {
    if (!h) return false;
    for (int i = 0; i < 8; ++i) s.s[i] = h[i];
    return true;
}

int gwfa_mlp_grad_dev(gwfa_ctx* ctx, const float* d_feat, int64_t n, int64_t feat_stride, const uint8_t* d_label,
                      const float* feat_scale, float pos_weight, const uint16_t* d_w, float* d_grad, float* d_loss,
                      void* hip_stream) {
    Scale8 sc;
    if (!ctx || n < 0 || feat_stride < 8 || !get_scale(feat_scale, sc) || !d_w || !d_grad || !d_loss ||
        !(pos_weight > 0.0f))
        return GWFA_ERR_ARG;
    if (n > 0 && (!d_feat || !d_label)) return GWFA_ERR_ARG;
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if (!ctx->d_mlp_scr)
        if (hipMalloc((void**)&ctx->d_mlp_scr, (size_t)gwfa_mlp_scratch_floats(MLP_SCR_SAMPLES) * 4) != hipSuccess) {
            ctx->d_mlp_scr = nullptr;
            return GWFA_ERR_NOMEM;
        }
    HIPCHK(ctx, gwfa_launch_mlp_grad(d_feat, feat_stride, sc, d_label, n, pos_weight, d_w, ctx->d_mlp_scr,
                                     MLP_SCR_SAMPLES, d_grad, d_loss, st));
    return GWFA_OK;
}

int gwfa_mlp_adam_dev(gwfa_ctx* ctx, float* d_master, float* d_m1, float* d_m2, const float* d_grad, uint16_t* d_w,
                      int32_t step, float lr, float beta1, float beta2, float eps, void* hip_stream) {
    if (!ctx || !d_master || !d_m1 || !d_m2 || !d_grad || !d_w || step < 1) return GWFA_ERR_ARG;
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return GWFA_ERR_ARG;
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const float bc1 = 1.0f - (float)std::pow((double)beta1, (double)step);
    const float bc2 = 1.0f - (float)std::pow((double)beta2, (double)step);
    HIPCHK(ctx, gwfa_launch_mlp_adam(d_master, d_m1, d_m2, d_grad, d_w, lr, beta1, beta2, eps, bc1, bc2, st));
    return GWFA_OK;
}

int gwfa_mlp_cast_dev(gwfa_ctx* ctx, const float* d_src, uint16_t* d_dst, int64_t n, void* hip_stream) {
    if (!ctx || n < 0 || (n > 0 && (!d_src || !d_dst))) return GWFA_ERR_ARG;
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, gwfa_launch_mlp_cast(d_src, d_dst, n, st));
    return GWFA_OK;
}

int gwfa_mlp_logits_dev(gwfa_ctx* ctx, const float* d_feat, int64_t n, int64_t feat_stride, const float* feat_scale,
                        const uint16_t* d_w, float* d_out, void* hip_stream) {
    Scale8 sc;
    if (!ctx || n < 0 || feat_stride < 8 || !get_scale(feat_scale, sc) || !d_w) return GWFA_ERR_ARG;
    if (n > 0 && (!d_feat || !d_out)) return GWFA_ERR_ARG;
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, gwfa_launch_mlp_logits(d_feat, feat_stride, sc, n, d_w, d_out, st));
    return GWFA_OK;
}

int gwfa_stats(gwfa_ctx* ctx, int64_t* out16, int32_t reset) {
    if (!ctx || !out16) return GWFA_ERR_ARG;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    unsigned long long h[16];
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(h, ctx->d_stats, sizeof(h), hipMemcpyDeviceToHost));
    for (int i = 0; i < 16; ++i) out16[i] = (int64_t)h[i];
    out16[5] = ctx->rerun_total;
    if (reset) {
        HIPCHK(ctx, hipMemset(ctx->d_stats, 0, sizeof(h)));
        ctx->rerun_total = 0;
    }
    return GWFA_OK;
}

}  // extern "C"
