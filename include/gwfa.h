/*
 * gwfa.h -- C ABI of the MI355X (gfx950) graph wavefront alignment library.
 *
 * The library aligns queries (DNA strings over A,C,G,T) to a sequence graph
 * whose vertices carry strings and whose directed edges may form cycles
 * (Section 2.1, Definitions 2.1 and 2.2 of Zhang, Wu, Aluru and Li, "Fast
 * sequence to graph alignment using the graph wavefront algorithm").  For
 * each query it returns the unit-cost edit distance of Eq. 1 (Section 2.2),
 * the end position, and the vertex walk (Section 2.6, Algorithms 5-6).
 *
 * Problem forms.  Extension mode (opts.end_vertex = -1): the walk starts
 * before the first base of the start vertex, the whole query is consumed,
 * the end is free anywhere in the graph.  The distance is the minimum of
 * Eq. 1 over the last query row; the end (end_v, end_off) is the
 * lexicographically smallest cell of that row holding the minimum, counting
 * cells with end_off >= 1 plus the start cell (start vertex, 0).  end_off is
 * the number of bases of end_v consumed.
 * Global form (Definition 2.2 as printed, Algorithm 1's end test): the walk
 * runs from before the first base of the start vertex to the last base of an
 * end vertex v_e; the distance is Eq. 1 at the cell (|q|, v_e, |v_e|) and
 * the end is (v_e, |v_e|).  One end vertex for every query
 * (opts.end_vertex >= 0) or one per query (gwfa_align_global_dev).
 * Start offset (either form, gwfa_align_at_dev): the walk starts after the
 * first j0 bases of the start vertex, i.e. Eq. 1's initial condition moves
 * to the cell (0, v_s, j0) -- a read seeded inside a vertex.  The start cell
 * is then (v_s, j0), and (v_s, 0) is no end cell when j0 > 0.
 *
 * Conventions for every call:
 *   - every int-returning call returns GWFA_OK (0) or a negative GWFA_ERR_*;
 *     outputs are defined only on GWFA_OK; no call aborts the process;
 *   - "host" pointers are CPU memory, "device" pointers are HIP device memory
 *     on the context's device; sizes are element counts unless stated;
 *   - a context is used by one host thread at a time; a graph is immutable
 *     after creation and may be shared by contexts on the same device.
 */
#ifndef GWFA_H
#define GWFA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define GWFA_OK               0
#define GWFA_ERR_ARG         -1   /* null pointer, negative size, bad option   */
#define GWFA_ERR_VERTEX      -2   /* start vertex or edge endpoint out of range */
#define GWFA_ERR_ALPHABET    -3   /* a base outside ACGT/acgt                   */
#define GWFA_ERR_EMPTY_LABEL -4   /* a vertex with an empty string              */
#define GWFA_ERR_NOMEM       -5   /* host or device allocation failed           */
#define GWFA_ERR_DEVICE      -6   /* a HIP call failed (see gwfa_last_error)    */
#define GWFA_ERR_PATH_CAP    -7   /* path buffer too small; distances valid     */
#define GWFA_ERR_UNSUPPORTED -8   /* option not available (see each call)       */
#define GWFA_ERR_FORMAT      -9   /* malformed GFA text (see gwfa_gfa_parse)     */

/* ---- per-query status (gwfa_result.status) ----------------------------- */
#define GWFA_ST_OK        0
#define GWFA_ST_MAX_SCORE 1       /* stopped at opts.max_score without an end  */
#define GWFA_ST_ARENA     2       /* the per-query working memory overflowed at
                                     every size tier tried                      */
#define GWFA_ST_BAD_INPUT 3       /* start (or end) vertex out of range         */
#define GWFA_ST_UNREACHABLE 4     /* global form: no walk from the start vertex
                                     reaches the end vertex                     */

/* ---- pruning modes (gwfa_opts.prune) ----------------------------------- */
#define GWFA_PRUNE_NONE      0    /* exact: Algorithms 1-3                      */
#define GWFA_PRUNE_HEURISTIC 1    /* Algorithm 4 before each expansion          */
#define GWFA_PRUNE_LEARNED   2    /* MLP keep/drop per diagonal before each
                                     expansion (needs gwfa_mlp_load, else
                                     GWFA_ERR_UNSUPPORTED)                      */

typedef struct gwfa_ctx gwfa_ctx;       /* device, stream, working memory    */
typedef struct gwfa_graph gwfa_graph;   /* packed labels + out-edge CSR      */

typedef struct {
    int32_t prune;          /* GWFA_PRUNE_*                                        */
    int32_t a_diff;         /* heuristic: drop a diagonal when a_max - a >= a_diff,
                               with a = query bases aligned + walk bases aligned
                               (Algorithm 4); must be >= 1 when prune = 1          */
    float keep_threshold;   /* learned: keep when the MLP logit >= keep_threshold   */
    int32_t traceback;      /* 1: fill walks (Algorithms 5-6); 0: distances only     */
    int32_t max_score;      /* -1: unbounded; else stop a query past this score     */
    int32_t end_vertex;     /* -1: extension mode; >= 0: global form, this end vertex
                               for every query (GWFA_ERR_VERTEX if out of range) */
    int32_t mlp_gate;       /* learned: run the MLP only when |F_s| >= mlp_gate     */
    int32_t mlp_period;     /* learned: run the MLP every mlp_period scores (>= 1)  */
    int32_t query_end_free; /* free end gap in the query: up to this many trailing
                               bases may stay unaligned at no cost (soft clip);
                               the distance is then the best over query prefixes
                               of at least |q| - query_end_free bases, ties to the
                               longest; 0: the whole query is aligned, as in
                               Definition 2.2, which penalises the query's end
                               gaps (>= 0; values above |q| act as |q|)            */
    int32_t walk_end_free;  /* global form: 1 lets the walk end anywhere inside the
                               end vertex (a free end gap in the walk, one of the
                               variants Section 2.2 points to): the best cell
                               (|q|, v_e, j) over j >= 1, plus j = 0 when v_e is
                               the start vertex and the walk starts at offset 0;
                               the smallest j on ties.  0: the walk ends at the
                               last base of v_e (Definition 2.2).  No effect in
                               extension mode, whose end is already free (0/1) */
} gwfa_opts;

typedef struct {
    int32_t dist;           /* edit distance d*, -1 unless status == GWFA_ST_OK   */
    int32_t end_v;          /* end vertex                                          */
    int32_t end_off;        /* bases of end_v consumed, 1..|end_v| (0 only for the
                               start vertex with start offset 0)                   */
    int32_t status;         /* GWFA_ST_*                                           */
    int64_t path_off;       /* first vertex of the walk in path_buf, -1 if none    */
    int32_t path_len;       /* vertices in the walk (start ... end_v)              */
    int32_t n_scores;       /* scores run (dist + 1 on success)                    */
    int64_t work;           /* sum over scores s of |F_s| (entries after extension) */
    int64_t t_begin;        /* device wall clock (100 MHz ticks) when the query   */
    int64_t t_end;          /* was taken from the work queue / finished           */
    int32_t start_off;      /* bases of the walk's first vertex skipped (the start
                               offset, or where in its start window the traced
                               walk starts; 0 by default)                           */
    int32_t clip;           /* trailing query bases left unaligned (at most
                               opts.query_end_free; 0 by default)                  */
} gwfa_result;              /* 64 bytes */

/* Default options: exact, traceback on, unbounded, extension mode. */
void gwfa_opts_default(gwfa_opts *opts);

/* Error text for a GWFA_ERR_* code (static storage). */
const char *gwfa_strerror(int code);

/* Last device-side error message kept in the context ("" if none). */
const char *gwfa_last_error(const gwfa_ctx *ctx);

/* Creates a context on HIP device `device`.  `hip_stream` is a hipStream_t on
 * that device, or NULL for the HIP null stream (which orders with every
 * blocking stream of the device); the library never destroys a stream.
 * Working memory is allocated (and cleared, synchronously) on the first
 * alignment call. */
int gwfa_ctx_create(int device, void *hip_stream, gwfa_ctx **out);
void gwfa_ctx_destroy(gwfa_ctx *ctx);

/* Working-memory / launch configuration (used by the autotuner).
 *   lanes_per_query: 64, 128, 256 or 512 threads cooperate on one query;
 *   n_groups: persistent workgroups (0 = as many as can be resident on the
 *             device at once for the chosen lanes_per_query);
 *   dir_log2_max: log2 of the largest per-query diagonal-page directory
 *                 (each page holds 32 diagonals of one vertex; 10..22);
 *   list_cap: capacity of each per-query wavefront list (entries, even);
 *   dir_factor: initial directory slots per 32 query bases (power of two).
 * Returns GWFA_ERR_ARG on a value out of range.  Frees working memory, which
 * is reallocated on the next call. */
int gwfa_ctx_config(gwfa_ctx *ctx, int32_t lanes_per_query, int32_t n_groups,
                    int32_t dir_log2_max, int32_t list_cap, int32_t dir_factor);

/* Builds a graph (Definition 2.1).  Host inputs, copied; the caller may free
 * them on return.
 *   seq      ASCII labels of all vertices concatenated (A,C,G,T, any case);
 *   seq_off  n_vtx+1 offsets into seq, non-decreasing; |v| = seq_off[v+1] -
 *            seq_off[v] must be >= 1 (GWFA_ERR_EMPTY_LABEL);
 *   edge_src, edge_dst  n_edge directed edges (u, v), 0 <= u, v < n_vtx
 *            (GWFA_ERR_VERTEX); self-loops and repeated edges are allowed.
 * The labels are packed 2 bits per base (A0 C1 G2 T3, first base in the most
 * significant bits, 32 bases per 64-bit word) and the edges are stored as an
 * out-edge CSR in device memory. */
int gwfa_graph_create(gwfa_ctx *ctx, int32_t n_vtx, const uint8_t *seq, const int64_t *seq_off,
                      int64_t n_edge, const int32_t *edge_src, const int32_t *edge_dst,
                      gwfa_graph **out);
void gwfa_graph_destroy(gwfa_graph *g);

/* Packs n_bases ASCII bases (device) into 2-bit words (device, at least
 * gwfa_packed_words(n_bases) words: the 2-word zero tail is written too) on
 * `hip_stream` (NULL = the context's stream).  A base outside ACGT/acgt sets
 * *d_err (device int32, the caller clears it first) to GWFA_ERR_ALPHABET;
 * the packed words are then unspecified.  Asynchronous. */
int gwfa_pack_dev(gwfa_ctx *ctx, const uint8_t *d_ascii, int64_t n_bases, uint64_t *d_packed,
                  int32_t *d_err, void *hip_stream);
int64_t gwfa_packed_words(int64_t n_bases);

/* Aligns n_reads queries (host buffers).
 *   reads     ASCII queries concatenated; read_off n_reads+1 offsets (bases);
 *   v_start   start vertex per query;
 *   res       n_reads results (host, caller-owned);
 *   path_buf  host buffer of path_cap vertex ids for the walks (may be NULL
 *             when opts->traceback == 0); *path_needed receives the number of
 *             ids the walks need (may be NULL).
 * Validates everything (ALPHABET, VERTEX, ARG) before any device work.
 * Returns GWFA_ERR_PATH_CAP when the walks do not fit; distances and ends are
 * then valid and the walks' path_off are -1.  Synchronous. */
int gwfa_align_batch(gwfa_ctx *ctx, const gwfa_graph *g, int32_t n_reads, const uint8_t *reads,
                     const int64_t *read_off, const int32_t *v_start, const gwfa_opts *opts,
                     gwfa_result *res, int32_t *path_buf, int64_t path_cap, int64_t *path_needed);

/* One query (host buffers): q (qlen ASCII bases) from start vertex v_start
 * (Definition 2.2, Algorithm 1's distance and Algorithm 6's walk).  The same
 * as gwfa_align_batch with one query; on GWFA_ERR_PATH_CAP, res->path_len is
 * the number of ids the walk needs.  Synchronous. */
int gwfa_align(gwfa_ctx *ctx, const gwfa_graph *g, const uint8_t *q, int32_t qlen, int32_t v_start,
               const gwfa_opts *opts, gwfa_result *res, int32_t *path_buf, int64_t path_cap);

/* The same on device-resident inputs (the form the Python binding uses).
 *   d_packed   packed queries (gwfa_pack_dev layout, 2-word zero tail);
 *   d_read_off n_reads+1 int64 base offsets; d_v_start n_reads int32;
 *   d_order    optional int32 permutation of 0..n_reads-1 giving the order in
 *              which queries are taken from the work queue (NULL = 0,1,2,...;
 *              longest first balances the load best);
 *   d_res      n_reads gwfa_result; d_path_buf path_cap int32 (may be NULL);
 *   d_path_used  device int64: receives the ids the walks need.
 * Per-query parameters are checked on the device by a screen pass before
 * the alignment kernel: a query whose start vertex is out of range gets its
 * result there (status GWFA_ST_BAD_INPUT) and never enters the alignment.
 * Runs on `hip_stream` (NULL = context stream).  When some query overflows its
 * working memory the library synchronises the stream and re-runs those
 * queries with larger memory before returning; otherwise the call is
 * asynchronous.  Returns GWFA_ERR_PATH_CAP only from gwfa_align_batch (here
 * the caller compares *d_path_used with path_cap). */
int gwfa_align_batch_dev(gwfa_ctx *ctx, const gwfa_graph *g, int32_t n_reads, const uint64_t *d_packed,
                         const int64_t *d_read_off, const int32_t *d_v_start, const int32_t *d_order,
                         const gwfa_opts *opts, gwfa_result *d_res, int32_t *d_path_buf, int64_t path_cap,
                         int64_t *d_path_used, void *hip_stream);

/* Global form with one end vertex per query: d_v_end (device, n_reads
 * int32).  Everything else as gwfa_align_batch_dev (opts.end_vertex must be
 * -1).  A query whose end vertex is out of range gets GWFA_ST_BAD_INPUT; one
 * whose end vertex cannot be reached gets GWFA_ST_UNREACHABLE (which may take
 * as long as exploring every cell reachable from its start; opts.max_score
 * bounds it). */
int gwfa_align_global_dev(gwfa_ctx *ctx, const gwfa_graph *g, int32_t n_reads, const uint64_t *d_packed,
                          const int64_t *d_read_off, const int32_t *d_v_start, const int32_t *d_v_end,
                          const int32_t *d_order, const gwfa_opts *opts, gwfa_result *d_res,
                          int32_t *d_path_buf, int64_t path_cap, int64_t *d_path_used, void *hip_stream);

/* Both forms with per-query start offsets: d_start_off (device, n_reads
 * int32, or NULL for all 0) gives j0, 0 <= j0 <= |v_start|, the bases of the
 * start vertex before the walk's start; d_start_hi (device, n_reads int32,
 * or NULL for j1 = j0; needs d_start_off) gives j1, j0 <= j1 <= |v_start|:
 * the walk may start after any j in j0..j1 bases at no cost (Eq. 1 with
 * H(0, v_start, j) = 0 across the window: a free leading gap in the start
 * vertex); d_v_end (device, n_reads int32) the end vertices of the global
 * form, or NULL for opts.end_vertex (then -1 is extension mode).  A query
 * whose start window or end vertex is out of range gets GWFA_ST_BAD_INPUT.
 * The walk written for a query begins with its start vertex;
 * gwfa_result.start_off is the offset the traced walk starts after (j0 when
 * traceback is off).  The cell (v_start, 0) ends a walk only when j0 = 0.
 * Everything else as gwfa_align_batch_dev. */
int gwfa_align_at_dev(gwfa_ctx *ctx, const gwfa_graph *g, int32_t n_reads, const uint64_t *d_packed,
                      const int64_t *d_read_off, const int32_t *d_v_start, const int32_t *d_start_off,
                      const int32_t *d_start_hi, const int32_t *d_v_end, const int32_t *d_order,
                      const gwfa_opts *opts, gwfa_result *d_res, int32_t *d_path_buf, int64_t path_cap,
                      int64_t *d_path_used, void *hip_stream);

/* The same, also writing one trace record per wavefront entry of every
 * score that is expanded (all scores before the final one), taken after the
 * extension and any pruning of that score, just before the expansion: the
 * training data of the learned pruning network.  Record r of d_dump
 * (device, 16 x 4 bytes, dump_cap records) holds
 *   float f[8]   the entry's eight features before scaling (the inputs of
 *                the network, see gwfa_mlp_load);
 *   int32 read, score s, i, v, off, W (walk bases), k (= i - off), attempt.
 * (i, v, off) is the entry's front cell: i query bases and off bases of v
 * consumed (Eq. 2).  A query that restarts with more working memory writes
 * its records again with a larger `attempt`; only the records of the largest
 * attempt of a query belong to its final run.  *d_dump_count (device int64,
 * cleared by the call) receives the number of records produced; those past
 * dump_cap are not written.  Slower than gwfa_align_batch_dev; asynchronous
 * under the same rule. */
int gwfa_align_dump_dev(gwfa_ctx *ctx, const gwfa_graph *g, int32_t n_reads, const uint64_t *d_packed,
                        const int64_t *d_read_off, const int32_t *d_v_start, const int32_t *d_order,
                        const gwfa_opts *opts, gwfa_result *d_res, int32_t *d_path_buf, int64_t path_cap,
                        int64_t *d_path_used, float *d_dump, int64_t dump_cap, int64_t *d_dump_count,
                        void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same as
 * gwfa_align_batch_dev, but the call allocates nothing and never waits on the
 * host.  Its working memory is a static array of 512 MiB in the library's
 * device code, one per device, held from the library's first use on that
 * device (the first context created there clears it) until the process
 * ends; it holds one fixed tier of working memory (record directory of 2^14
 * pages and wavefront lists of 8,192 entries per query), so a query that
 * outgrows it gets GWFA_ST_ARENA and is not re-run (gwfa_align_batch_dev
 * re-runs such queries with more memory).  At most 2^20 queries per call
 * (GWFA_ERR_ARG beyond, with the reason in gwfa_last_error).  Launches
 * kernels only (queue reset, screen pass, alignment) on `hip_stream`.  Every
 * call on one device shares that device's array: calls that overlap in time
 * on one device (from any context or thread) race and must not be issued.
 * GWFA_ERR_DEVICE if the array could not be set up on this device. */
int gwfa_align_batch_static_dev(gwfa_ctx *ctx, const gwfa_graph *g, int32_t n_reads, const uint64_t *d_packed,
                                const int64_t *d_read_off, const int32_t *d_v_start, const int32_t *d_order,
                                const gwfa_opts *opts, gwfa_result *d_res, int32_t *d_path_buf, int64_t path_cap,
                                int64_t *d_path_used, void *hip_stream);

/* Base-level alignment of each query against the walk it was aligned to: the
 * step that turns the walk of Algorithm 6 into an alignment (the paper leaves
 * it to a pairwise aligner, noting that it is cheap).  Inputs are the device
 * results and walks of a finished alignment call on the same queries
 * (d_packed, d_read_off as given to it; d_res, d_path_buf as it filled them).
 * For query r whose walk was traced, an optimal global alignment of q (its
 * first |q| - clip bases) and the walk's string (labels of the walk, the
 * first one from start_off, the last one cut at end_off) is written
 * as CIGAR operations (length << 4 | op, op 7 '=', 8 'X', 1 'I' = query base
 * absent from the walk, 2 'D' = walk base absent from the query, then
 * 4 'S' = the clip trailing query bases left unaligned, when clip > 0) into
 * d_cigar (cigar_cap words) at d_cigar_off[r], d_cigar_len[r] operations.
 * Its cost (X + I + D) is the walk's edit distance: the distance for exact
 * alignments, at most the distance under pruning.  d_cigar_len[r] = -1: no
 * walk (status not OK or traceback off); -2: d_cigar too small
 * (*d_cigar_used, device int64, receives the words needed); -3: internal
 * capacity.  Synchronises the stream once to size its working memory, then
 * runs asynchronously. */
int gwfa_cigar_dev(gwfa_ctx *ctx, const gwfa_graph *g, int32_t n_reads, const uint64_t *d_packed,
                   const int64_t *d_read_off, const gwfa_result *d_res, const int32_t *d_path_buf,
                   uint32_t *d_cigar, int64_t cigar_cap, int64_t *d_cigar_off, int32_t *d_cigar_len,
                   int64_t *d_cigar_used, void *hip_stream);

/* ---- GFA input ----------------------------------------------------------
 * Reads a sequence graph from GFA 1 text, the format pangenome graphs are
 * distributed in, into the arguments of gwfa_graph_create (Definition 2.1:
 * vertices labelled by strings, directed edges).  Host memory only: these
 * calls touch no device and need no context.
 *   S <name> <sequence> ...     a segment; the sequence is over ACGT/acgt
 *   L <a> <+|-> <b> <+|-> <overlap> ...   a link between oriented segments
 * Other record types are ignored.  Segment i (in file order) becomes vertex
 * 2i, its sequence, and vertex 2i+1, its reverse complement; a link
 * (a, oa, b, ob) becomes the edge a^oa -> b^ob and its complement
 * b^(-ob) -> a^(-oa), the same adjacency read on the other strand.  With
 * flags = GWFA_GFA_FORWARD, segment i is vertex i and only links + + are
 * kept (the others are counted in n_skipped).  Repeated edges are merged;
 * edges are sorted by (source, target).  Errors (with *err_line, 1-based,
 * when not NULL): GWFA_ERR_FORMAT for a malformed S or L record, a repeated
 * segment name or no segment at all; GWFA_ERR_ALPHABET for a base outside
 * ACGT; GWFA_ERR_EMPTY_LABEL for an empty sequence; GWFA_ERR_UNSUPPORTED for
 * a sequence given as '*' or an overlap other than '*' or 0M; GWFA_ERR_VERTEX
 * for a link naming an unknown segment; GWFA_ERR_ARG for an unreadable file
 * or bad arguments. */
#define GWFA_GFA_FORWARD 1
typedef struct gwfa_gfa gwfa_gfa;
int gwfa_gfa_load(const char *path, int32_t flags, gwfa_gfa **out, int64_t *err_line);
int gwfa_gfa_parse(const char *text, int64_t len, int32_t flags, gwfa_gfa **out, int64_t *err_line);
/* Sizes of the graph (any pointer may be NULL). */
int gwfa_gfa_sizes(const gwfa_gfa *g, int32_t *n_vtx, int64_t *n_bases, int64_t *n_edge, int32_t *n_segments,
                   int64_t *n_skipped);
/* Copies the graph into caller buffers of the sizes above: seq (n_bases
 * bytes), seq_off (n_vtx + 1), edge_src and edge_dst (n_edge each). */
int gwfa_gfa_graph(const gwfa_gfa *g, uint8_t *seq, int64_t *seq_off, int32_t *edge_src, int32_t *edge_dst);
/* Vertex of segment `name` in orientation reverse (0: as given, 1: reverse
 * complement); GWFA_ERR_VERTEX if there is none. */
int32_t gwfa_gfa_vertex(const gwfa_gfa *g, const char *name, int32_t reverse);
/* Segment name of vertex v (storage owned by g) and its orientation in
 * *reverse; NULL if v is out of range. */
const char *gwfa_gfa_name(const gwfa_gfa *g, int32_t v, int32_t *reverse);
void gwfa_gfa_free(gwfa_gfa *g);

/* ---- captured launches ---------------------------------------------------
 * A plan records the alignment of one device-resident batch (the arguments
 * of gwfa_align_batch_dev, fixed at creation) as a HIP graph: the reset of
 * the work queue and counters, the screen pass of the query parameters and
 * the first-tier launch of the persistent alignment kernel, kernels only.  gwfa_plan_launch replays it on
 * `hip_stream` (NULL = context stream), asynchronously, with no host work.
 * gwfa_plan_finish then synchronises that stream and re-runs, eagerly, the
 * queries that overflowed the first tier's working memory (usually none);
 * after it returns, results are complete exactly as after
 * gwfa_align_batch_dev.  The buffers named at creation must stay allocated;
 * gwfa_ctx_config invalidates the plan (its calls then return GWFA_ERR_ARG),
 * and so does a later call on the context with more queries than any before
 * (it moves the context's per-query lists);
 * destroy plans before their context.  Replays of one plan, like calls on one
 * context, must not overlap in time. */
typedef struct gwfa_plan gwfa_plan;
int gwfa_plan_create(gwfa_ctx *ctx, const gwfa_graph *g, int32_t n_reads, const uint64_t *d_packed,
                     const int64_t *d_read_off, const int32_t *d_v_start, const int32_t *d_order,
                     const gwfa_opts *opts, gwfa_result *d_res, int32_t *d_path_buf, int64_t path_cap,
                     int64_t *d_path_used, gwfa_plan **out);
int gwfa_plan_launch(gwfa_plan *plan, void *hip_stream);
int gwfa_plan_finish(gwfa_plan *plan, void *hip_stream);
void gwfa_plan_destroy(gwfa_plan *plan);

/* Loads the pruning network used with GWFA_PRUNE_LEARNED: 8 features ->
 * 64 ReLU -> 64 ReLU -> 1 logit, bfloat16 values in the order W1[64][8],
 * b1[64], W2[64][64], b2[64], W3[64], b3 (4801 values), plus 8 float
 * feature scales.  The network reads x = bf16(f * scale) for the features
 *   f0 log1p(a_max - a)  (a = i + W, Algorithm 4)   f1 log1p(s)
 *   f2 log1p(outdeg v)   f3 log1p(i_max - i)         f4 log1p(|v| - off)
 *   f5 sign(W - i) log1p(|W - i|)   f6 i / |q|       f7 log1p(|q| - i)
 * rounds each ReLU output to bfloat16 and sums in float32.  A diagonal is
 * kept when its logit >= opts.keep_threshold; the diagonal with the largest
 * a is always kept, and dropped diagonals keep their records (as in
 * Algorithm 4).  Host pointers, copied. */
int gwfa_mlp_load(gwfa_ctx *ctx, const uint16_t *bf16_weights, int64_t n, const float *feat_scale);

/* ---- training of the pruning network (device buffers, asynchronous on
 * `hip_stream`, NULL = context stream) ---------------------------------- */

/* Mean gradient and mean loss of n samples: features d_feat (float, row r at
 * d_feat + r * feat_stride, first 8 used, feat_stride >= 8), labels d_label
 * (uint8, nonzero = keep), feat_scale (host, 8 floats), weights d_w (4801
 * bfloat16).  Loss: binary cross-entropy on the logit, positives weighted by
 * pos_weight > 0.  The forward pass is the alignment kernel's inference
 * arithmetic; the backward pass treats the bfloat16 roundings as identities.
 * Overwrites d_grad (4801 floats) and *d_loss (float). */
int gwfa_mlp_grad_dev(gwfa_ctx *ctx, const float *d_feat, int64_t n, int64_t feat_stride, const uint8_t *d_label,
                      const float *feat_scale, float pos_weight, const uint16_t *d_w, float *d_grad, float *d_loss,
                      void *hip_stream);

/* One Adam step (step >= 1 is the 1-based step count used for the bias
 * corrections) on float32 master weights d_master with moments d_m1, d_m2
 * (4801 floats each); writes the bfloat16 copy d_w. */
int gwfa_mlp_adam_dev(gwfa_ctx *ctx, float *d_master, float *d_m1, float *d_m2, const float *d_grad,
                      uint16_t *d_w, int32_t step, float lr, float beta1, float beta2, float eps, void *hip_stream);

/* Rounds n floats to bfloat16 (nearest, ties to even). */
int gwfa_mlp_cast_dev(gwfa_ctx *ctx, const float *d_src, uint16_t *d_dst, int64_t n, void *hip_stream);

/* Logits of n samples computed by the alignment kernel's inference routine. */
int gwfa_mlp_logits_dev(gwfa_ctx *ctx, const float *d_feat, int64_t n, int64_t feat_stride, const float *feat_scale,
                        const uint16_t *d_w, float *d_out, void *hip_stream);

/* Training labels (host computation, no device needed).  For trace records
 * of exact runs (gwfa_align_dump_dev with GWFA_PRUNE_NONE) gives, per entry e
 * with front cell (ent_i, ent_v, ent_off) of query ent_read at score
 * ent_score, the cost out_cost[e] of the best completion of the alignment
 * from that cell (Eq. 1 read from the end of the query; the end is free), and
 * out_label[e] = [ent_score + out_cost = d*] (may be NULL): the entry lies on
 * an optimal alignment.  out_dist[r] receives d* of query r.  The graph and
 * queries are given as for gwfa_graph_create and gwfa_align_batch (host).
 * Memory: two rows of (bases + n_vtx) int32 per thread.  n_threads <= 0: all
 * hardware threads.  Returns GWFA_ERR_ARG for an entry outside its query or
 * vertex. */
int gwfa_label_entries(int32_t n_vtx, const uint8_t *seq, const int64_t *seq_off, int64_t n_edge,
                       const int32_t *edge_src, const int32_t *edge_dst, int32_t n_reads, const uint8_t *reads,
                       const int64_t *read_off, const int32_t *v_start, int64_t n_ent, const int32_t *ent_read,
                       const int32_t *ent_score, const int32_t *ent_i, const int32_t *ent_v, const int32_t *ent_off,
                       int32_t *out_cost, uint8_t *out_label, int32_t *out_dist, int32_t n_threads);

/* Kernel-level counters accumulated since the last reset (device totals over
 * every query): [0] wavefront entries (sum |F_s|), [1] crossings admitted,
 * [2] pages created, [3] 32-base compare chunks in the extension,
 * [4] expansion candidates admitted, [5] queries re-run for memory,
 * [6] MLP evaluations, [7] entries dropped by pruning, [8] scores run,
 * [9]..[12] device wall-clock ticks (100 MHz) summed over queries spent in
 * the expansion+extension pass, the crossing rounds, the crossing merge and
 * the pruning pass, [13]..[15] reserved.  out16 receives 16 values. */
int gwfa_stats(gwfa_ctx *ctx, int64_t *out16, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* GWFA_H */
