/*
 * libuhnsw -- the U-HNSW query path on one AMD Instinct MI355X (gfx950).
 *
 * Problem (U-HNSW paper, Wang, Meng, Xu, EDBT'27; Sec. 1.1 and Sec. 2.1):
 * each query is a tuple (q, p) with its own K; the answer is the top-K of
 * the dataset under the L_p distance d_p(x, q) = (sum_i |x_i - q_i|^p)^(1/p),
 * p in [0.5, 2]. Method (Sec. 3.1, Algorithm 1): pick G1 (an HNSW graph
 * built under L1) when p <= 1.4, else G2 (under L2); run HNSW's KnnSearch on
 * it to get t candidates C ordered by the base metric; verify C in batches
 * of kappa under L_p and stop once |R_new n R| / K >= tau. The extended
 * variant (Sec. 4.5) serves p in [0.2, 1] with G_0.5 (built under L0.5) in
 * G1's place, G_1 (under L1) in G2's, and a cutoff of 0.6.
 *
 * Conventions for every entry point:
 *   - plain C; no exception crosses the boundary;
 *   - return 0 (UHNSW_OK) or a negative UHNSW_E* code; on error nothing is
 *     written to any output and uhnsw_last_error(ctx) describes the failure;
 *   - the caller owns every array it passes; the library copies what it
 *     keeps (the index) and owns all device memory it allocates;
 *   - one context may be used by one host thread at a time.
 */
#ifndef UHNSW_H
#define UHNSW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UHNSW_OK 0
#define UHNSW_EINVAL (-1)      /* bad argument (NULL, size, range)            */
#define UHNSW_ENOMEM (-2)      /* host or device allocation failed            */
#define UHNSW_EDEVICE (-3)     /* a HIP call failed; context is now failed    */
#define UHNSW_ESTATE (-4)      /* search before load, or failed context       */
#define UHNSW_EIO (-5)         /* reserved for file loaders                   */
#define UHNSW_EBUSY (-6)       /* admission budget exhausted (serving)        */
#define UHNSW_EUNSUPPORTED (-7)/* shape the kernels were not built for        */

#define UHNSW_MAX_LAYERS 32
#define UHNSW_KMAX 256         /* largest K per query                          */
#define UHNSW_EFMAX 2048       /* largest efSearch per query (the paper goes
                                  to 2,000, Sec. 4.1.4)                        */
#define UHNSW_DMAX 1024        /* largest dimension                            */

/* Storage of the base vectors read by the candidate walk. Verification
 * always reads FP32 copies. */
#define UHNSW_STORE_F32 0
#define UHNSW_STORE_BF16 1     /* bfloat16, rounded to nearest even            */
#define UHNSW_STORE_F16 2      /* IEEE binary16, rounded to nearest even       */

/* per-query flag bits in uhnsw_stats.flags */
#define UHNSW_QBAD 1           /* query invalid (parameters, non-finite q):
                                  the row is left padded                      */
#define UHNSW_QCAP 2           /* walk stopped after n expansions (cannot
                                  happen for finite inputs; a safety bound)   */

typedef struct uhnsw_ctx uhnsw_ctx;

/* One HNSW graph as per-layer CSR (HNSW's layered proximity graph, Sec. 2.2).
 * Layer 0 holds every node 0..n-1: row_ptr[0] has n+1 entries. Layer l >= 1
 * holds the nodes with level >= l, listed ascending in nodes[l] (n_nodes[l]
 * of them); row_ptr[l] has n_nodes[l]+1 entries indexing col[l]. Degrees are
 * at most 2M on layer 0 and M above; neighbours of a layer-l node are on
 * layer l; entry_point has level max_level. All host pointers. */
typedef struct {
    int32_t M;
    int32_t max_level;
    int32_t entry_point;
    const int8_t *level;                          /* [n]                       */
    int64_t n_nodes[UHNSW_MAX_LAYERS];
    const int32_t *nodes[UHNSW_MAX_LAYERS];       /* layer >= 1                */
    const int64_t *row_ptr[UHNSW_MAX_LAYERS];
    const int32_t *col[UHNSW_MAX_LAYERS];
} uhnsw_graph;

/* Index variants (graph pair, base metrics, p range, default cutoff). */
#define UHNSW_VARIANT_STD 0    /* G1 under L1, G2 under L2; p in [0.5, 2];
                                  cutoff 1.4 (Sec. 3.1)                        */
#define UHNSW_VARIANT_EXT 1    /* G_0.5 under L0.5 (walk key sum sqrt|x - q|),
                                  G_1 under L1; p in [0.2, 1]; cutoff 0.6
                                  (Sec. 4.5)                                   */
#define UHNSW_VARIANT_PGRAPH 2 /* the per-p HNSW baseline (Sec. 4.3, Fig. 4):
                                  graphs[0] = G_p built for graph_p, walked
                                  under sum |x - q|^graph_p (v_log / v_exp);
                                  graphs[1] under L2 (only for p above the
                                  cutoff); p in [0.2, 2]; cutoff +inf: every
                                  query walks G_p and is verified under its
                                  own p (a query of p = graph_p is HNSW on
                                  its own metric)                             */

/* The resident index: base vectors (host, n x d FP32 row-major) and the two
 * base graphs, graphs[0] = G1 (built under L1), graphs[1] = G2 (under L2);
 * for UHNSW_VARIANT_EXT graphs[0] = G_0.5 and graphs[1] = G_1. */
typedef struct {
    int64_t n;
    int32_t d;
    const float *base;
    int32_t storage;          /* UHNSW_STORE_* for the walk                   */
    uhnsw_graph graphs[2];
    int32_t variant;          /* UHNSW_VARIANT_*; 0 (zero-initialised) = STD  */
    float graph_p;            /* UHNSW_VARIANT_PGRAPH: the p graphs[0] was
                                 built for, in [0.2, 2]; ignored otherwise   */
} uhnsw_index;

/* Algorithm 1's parameters (Sec. 3.1) and execution knobs. */
typedef struct {
    double tau;               /* early-termination threshold, default 0.92    */
    float cutoff;             /* graphs[0] when p <= cutoff (FP32 compare);
                                 0 -> the index's default (1.4, or 0.6 for
                                 the extended variant); negative: EINVAL     */
    int32_t t;                /* candidates; 0 -> min(ef, 6K), else min(ef,t) */
    int32_t kappa;            /* batch size; 0 -> max(K, 2)                   */
    int32_t beam_width;       /* nodes expanded per walk step, 1 = HNSW       */
    int32_t early_abort;      /* exact partial-sum abort in verification: for
                                 rows of more than 256 dimensions the second
                                 half of a row is read only while its partial
                                 sum is at most the K-th best of R; shorter
                                 rows are always read whole                   */
    int32_t visited_slots;    /* LDS visited-cache slots; 0 -> the largest
                                 power of two in 1,024 .. 8,192 that keeps a
                                 wave's LDS within 11 KiB (8,192 above ef
                                 512)                                        */
    int32_t waves_per_block;  /* 0 -> 1                                       */
    int32_t persistent;       /* schedule of the queries over the waves:
                                 0: one wave per query by grid position;
                                 1: persistent launch, waves take queries
                                 from a work counter until none is left;
                                 2: as 1, after a pre-pass that descends
                                 every query and orders the queries by
                                 layer-0 entry distance, largest first (the
                                 long walks start first, the launch's tail
                                 shortens);
                                 3 (default): the pre-pass and order of 2
                                 on the grid of 0 (grid position k takes
                                 the k-th query of the order).
                                 Results do not change.                     */
    int32_t timing;           /* 1: record per-kernel times (uhnsw_last_timing)*/
    int32_t fused;            /* 1: walk and verification in one kernel, C
                                 kept in LDS (the batching form)             */
    int32_t graph;            /* 1: capture the launch sequence as a hipGraph
                                 on first use and replay it while the
                                 arguments stay the same                     */
    int32_t waves_per_cu;     /* persistent launch: resident waves per CU
                                 (0 = as many as fit)                        */
} uhnsw_params;

/* Per-query counters (the N_b / N_p of the paper's cost model, Eq. 1). */
typedef struct {
    int32_t graph;            /* 1 = graphs[0] (G1), 2 = graphs[1] (G2)       */
    int32_t n_b;              /* base-metric distances (descent + layer 0)    */
    int32_t n_exp;            /* layer-0 expansions                           */
    int32_t n_p;              /* L_p distances evaluated                      */
    int32_t batches;          /* verification batches taken                   */
    int32_t nc;               /* |C|                                          */
    int32_t flags;            /* UHNSW_QBAD, ...                              */
    int32_t entry0;           /* layer-0 start node (end of the descent)      */
    uint32_t t_begin;         /* device wall clock when the walk of this query
                                 started / when its verification ended: low
                                 32 bits of a counter running at
                                 hipDeviceAttributeWallClockRate kHz           */
    uint32_t t_end;
    int32_t n_up;             /* base distances of the upper-layer descent
                                 (part of n_b; the rest are layer 0's)        */
    int32_t n_cut;            /* L_p rows (of n_p) whose second half was not
                                 read: the partial-sum abort (early_abort,
                                 rows of more than 256 dimensions)            */
} uhnsw_stats;

/* Fill *prm with the defaults above. */
void uhnsw_default_params(uhnsw_params *prm);

/* Create a context on HIP device `device`. *out receives the handle.
 * Errors: EINVAL (out NULL, no such device), EDEVICE, ENOMEM. */
int uhnsw_create(int device, uhnsw_ctx **out);

/* Free the context and all device memory it owns. NULL is a no-op. With a
 * server still running on the context (uhnsw_serve_start without
 * uhnsw_serve_stop) nothing is freed and uhnsw_last_error says so: stop the
 * servers first. */
void uhnsw_destroy(uhnsw_ctx *ctx);

/* Message for the last failure on ctx (or of uhnsw_create when ctx is NULL).
 * The string is owned by the library and valid until the next call on ctx. */
const char *uhnsw_last_error(const uhnsw_ctx *ctx);

/* Recover a context that a device error (EDEVICE, or ENOMEM from a device
 * allocation) marked failed; a failed context answers every search with
 * ESTATE until this call or a successful uhnsw_load_graphs. Not an
 * operation of the method: it lets a caller that keeps one context for its
 * lifetime (a service answering query tuples as in the problem statement,
 * Sec. 1.1) go on after a failure. Waits for the device, then drops the
 * captured hipGraphs and all per-stream and staging scratch (reallocated on
 * next use); the loaded index stays. A context that is not failed is reset
 * the same way.
 * Errors: EINVAL (NULL), ESTATE (a server is running on the context),
 * EDEVICE (the device still reports an error: the context stays failed and
 * should be destroyed). */
int uhnsw_reset(uhnsw_ctx *ctx);

/* Validate the index and copy it to the device, replacing any loaded index.
 * Layer 0 becomes fixed-degree rows of 2M ids (-1 padded); upper layers get
 * M-wide rows addressed through a per-node offset; base vectors get a padded
 * row pitch (zeros) and, for BF16/F16 storage, a converted walk copy.
 * Errors: EINVAL (any structural violation: id out of range, degree above
 * 2M / M, neighbour not on the layer, a row listing one neighbour twice or
 * the node itself (a neighbour list is a set of other nodes, Sec. 2.2),
 * entry point not on the top layer, d > UHNSW_DMAX, M0 > 64, a non-finite
 * base value, an unknown variant, graph_p outside [0.2, 2] for
 * UHNSW_VARIANT_PGRAPH),
 * ESTATE (a server is running on the context), ENOMEM, EDEVICE. */
int uhnsw_load_graphs(uhnsw_ctx *ctx, const uhnsw_index *idx);

/* uhnsw_load_graphs from files (host paths):
 *   vec_path: base vectors, .fbin layout: int32 n, int32 d, then n*d FP32
 *             row-major (little-endian);
 *   g1_path / g2_path: graphs[0] / graphs[1] of `variant` (G1 / G2, or
 *             G_0.5 / G_1), layout:
 *             "UHG1", int32 n, int32 M, int32 max_level, int32 entry_point,
 *             int8 level[n], then for each layer l = 0 .. max_level:
 *             int64 n_l (n for l = 0), int64 row_ptr[n_l + 1],
 *             int32 col[row_ptr[n_l]], and for l >= 1 int32 nodes[n_l].
 * The files are read into host memory, checked as uhnsw_load_graphs checks
 * its arguments, uploaded, and released.
 * Errors: EIO (cannot open, short file, bad magic, n differs between
 * files), EINVAL (as uhnsw_load_graphs, or sizes out of range), ENOMEM,
 * EDEVICE. */
int uhnsw_load_graph_files(uhnsw_ctx *ctx, const char *vec_path, const char *g1_path, const char *g2_path,
                           int32_t storage, int32_t variant);

/* Host-only validation: the checks uhnsw_load_graphs (resp.
 * uhnsw_load_graph_files) makes before it touches a device, with no context
 * and no HIP call, so an index can be vetted on a machine without a GPU.
 * msg (may be NULL) receives the reason for a failure ("" on success),
 * NUL-terminated and cut to msg_len bytes; the index stays the caller's.
 * Returns UHNSW_OK, UHNSW_EINVAL (structure, as uhnsw_load_graphs) or, for
 * the files form, UHNSW_EIO (as uhnsw_load_graph_files). */
int uhnsw_check_index(const uhnsw_index *idx, char *msg, int32_t msg_len);
int uhnsw_check_index_files(const char *vec_path, const char *g1_path, const char *g2_path, int32_t storage,
                            int32_t variant, char *msg, int32_t msg_len);

/* Search nq queries (host arrays, synchronous).
 *   queries [nq x d] FP32; p [nq]; k [nq]; ef [nq]; prm may be NULL.
 *   ids [nq x k_stride] int64 and dists [nq x k_stride] FP32 receive, per
 *   row, min(k[i], |C_i|) results ascending by (L_p distance, id); the rest
 *   of the row is id -1, dist +inf. stats [nq] may be NULL.
 * Errors: EINVAL (NULL pointer, nq < 0, p not finite or outside the
 * index's range ([0.5, 2]; [0.2, 1] for UHNSW_VARIANT_EXT; [0.2, 2] for
 * UHNSW_VARIANT_PGRAPH),
 * k < 1 or > UHNSW_KMAX, ef < k or > UHNSW_EFMAX, k_stride < max k, a
 * non-finite query value),
 * ESTATE (no index), ENOMEM, EDEVICE. */
int uhnsw_search(uhnsw_ctx *ctx, const float *queries, int64_t nq, const float *p, const int32_t *k,
                 const int32_t *ef, const uhnsw_params *prm, int32_t k_stride, int64_t *ids, float *dists,
                 uhnsw_stats *stats);

/* Same search on device pointers, asynchronous on `stream` (a hipStream_t;
 * NULL = the null stream). The caller promises k[i] <= k_max and
 * ef[i] <= ef_max (host scalars sizing LDS); a query whose values break
 * this or the ranges above, or whose vector is not finite, is not searched:
 * its row is padded and its stats get UHNSW_QBAD. cand_ids / cand_keys (device, [nq x c_stride], may be
 * NULL) receive C and its base-metric keys (-1 / +inf padded). Buffers are
 * borrowed until the stream's work completes. Searches on different streams
 * may run at the same time: each stream gets its own scratch (candidate
 * lists, work counter, timing events, captured hipGraph) on first use, up to
 * 64 streams per context. Calls on one context from several host threads at
 * once are not supported.
 * Errors: EINVAL (host-checkable arguments), ESTATE, ENOMEM, EDEVICE,
 * EUNSUPPORTED (a 65th stream). */
int uhnsw_search_device(uhnsw_ctx *ctx, const float *queries, int64_t nq, const float *p, const int32_t *k,
                        const int32_t *ef, int32_t k_max, int32_t ef_max, const uhnsw_params *prm,
                        int32_t k_stride, int64_t *ids, float *dists, uhnsw_stats *stats, int32_t *cand_ids,
                        float *cand_keys, int32_t c_stride, void *stream);

/* uhnsw_search_device for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same search, arguments and results, but the call makes no device, pinned
 * or host allocation and creates no HIP object. Its scratch (default stats
 * when `stats` is NULL, the two-kernel form's candidate lists when
 * cand_ids is NULL, the work counter, the ordering pre-pass arrays) is
 * carved from one fixed region of UHNSW_NOALLOC_SCRATCH_BYTES per device,
 * reserved when the library's code object loads and held until the process
 * ends; the caller still passes inputs and outputs. Every call on one
 * device shares that region and it keeps the last call's contents (what
 * must start at zero is cleared by a kernel on `stream`), so calls that
 * overlap on one device race: serialise them (one stream, or wait between
 * streams). A search needs about nq x (44 + 20 + 4) bytes, plus
 * nq x ef_max x 8 for the two-kernel form without caller-held candidate
 * arrays; one that needs more than the region fails.
 * Errors: EINVAL (as uhnsw_search_device; also prm->graph or prm->timing
 * set, or scratch above the region), ESTATE, EDEVICE. */
#define UHNSW_NOALLOC_SCRATCH_BYTES (64ll << 20)
int uhnsw_search_device_noalloc(uhnsw_ctx *ctx, const float *queries, int64_t nq, const float *p, const int32_t *k,
                                const int32_t *ef, int32_t k_max, int32_t ef_max, const uhnsw_params *prm,
                                int32_t k_stride, int64_t *ids, float *dists, uhnsw_stats *stats,
                                int32_t *cand_ids, float *cand_keys, int32_t c_stride, void *stream);

/* Batching form: pick execution knobs for this index and query mix by
 * timing the search on the given device queries (same arrays and limits as
 * uhnsw_search_device): visited-cache slots, waves per block, the schedule
 * (persistent field), for a persistent winner the resident waves per CU
 * (8, 12 or as many as fit), and -- only with UHNSW_TUNE_BEAM in `flags`, since it changes the
 * walk's trajectory -- the beam width. Every other knob leaves results
 * unchanged. With UHNSW_TUNE_PIPELINED the knobs are timed as back-to-back
 * launches alternating between `stream` and a second stream of the
 * context (the throughput of a caller that keeps two batches in flight)
 * instead of one launch at a time. *prm is read for Algorithm 1's
 * parameters and receives the chosen knobs. Results are cached per (n, d,
 * storage, ef range, k_max, flags, fused, index variant) in the context.
 * Errors: EINVAL, ESTATE, ENOMEM, EDEVICE. */
#define UHNSW_TUNE_BEAM 1
#define UHNSW_TUNE_PIPELINED 2
int uhnsw_autotune(uhnsw_ctx *ctx, const float *queries, int64_t nq, const float *p, const int32_t *k,
                   const int32_t *ef, int32_t k_max, int32_t ef_max, int32_t flags, uhnsw_params *prm,
                   void *stream);

/* Number of hipGraph captures made so far (prm->graph); replays do not
 * count. */
int uhnsw_graph_captures(const uhnsw_ctx *ctx, int64_t *count);

/* Lane layout of the walk's FP32 base distance for the loaded index:
 * element j is summed by lane (j / v) mod g, lanes combine pairwise. */
int uhnsw_get_layout(const uhnsw_ctx *ctx, int32_t *g, int32_t *v);

/* Ceiling probes for reading the rooflines (measurement only, not part of
 * the query path; synchronous on the context's stream).
 * uhnsw_probe_gather: HBM rate, in GB/s (1e9 B/s), of random gathers of
 * `row_bytes` (128, 256 or 512) from the loaded FP32 rows with the walk's
 * access pattern (8 lanes per row, 16-B loads, 32 rows in flight per wave)
 * but no dependency between batches: the rate the walk's gathers could
 * reach at best. Row ids come from a fixed hash.
 * Errors: EINVAL (NULL, row_bytes not 128/256/512 or above the row pitch),
 * ESTATE (no index), ENOMEM, EDEVICE. */
int uhnsw_probe_gather(uhnsw_ctx *ctx, int32_t row_bytes, double *gbs);

/* uhnsw_probe_transcendental: v_exp_f32 + v_log_f32 lane operations per
 * second over independent chains on every CU (the unit the verification's
 * general-p power uses). Errors: EINVAL (NULL), ENOMEM, EDEVICE. */
int uhnsw_probe_transcendental(uhnsw_ctx *ctx, double *ops_per_s);

/* Device facts for callers that interpret uhnsw_stats: compute units and the
 * rate (kHz) of the wall clock behind t_begin / t_end. */
int uhnsw_device_info(const uhnsw_ctx *ctx, int32_t *num_cus, int32_t *wall_clock_khz);

/* Kernel times (ms) of the last search run with prm->timing = 1, measured
 * with HIP events on the stream the kernels ran on. walk_ms covers the
 * descent pre-pass (schedules 2, 3) and the walk kernel (the fused kernel,
 * verification included, with prm->fused); verify_ms the verification
 * kernel (0 with prm->fused). */
int uhnsw_last_timing(const uhnsw_ctx *ctx, float *walk_ms, float *verify_ms);

/* The same search's times split three ways: prepass_ms the descent pre-pass
 * and ordering kernels (0 without them), walk_ms the walk kernel alone (the
 * fused kernel with prm->fused), verify_ms the verification kernel. A search
 * replayed from a captured hipGraph has no split: ESTATE. */
int uhnsw_last_timing_split(const uhnsw_ctx *ctx, float *prepass_ms, float *walk_ms, float *verify_ms);

/* ------------------------------------------------- graph construction
 * GPU construction of one HNSW base graph (HNSW's layered graph, Sec. 2.2;
 * building G1 and G2 is the method's up-front cost, Sec. 4.4.3, Table 3)
 * under metric 1 (L1, for G1 and G_1), 2 (squared L2, for G2), 3
 * (sum sqrt|x - q|, for G_0.5) or 4 (sum |x - q|^metric_p, for the per-p
 * baseline's G_p; each term exp2(p log2|x - q|) on v_log / v_exp), on the
 * context's device:
 *   - node levels floor(-ln(U_v) / ln M) with U_v in (0, 1] from
 *     splitmix64(seed ^ v * 0x9E3779B97F4A7C15) (top 53 bits + 1) / 2^53,
 *     capped at 30;
 *   - insertion in id order, in batches of clamp(nodes in the graph / 64,
 *     1, batch_max) that are planned against the graph frozen at the batch
 *     start: greedy descent above the node's level, a best-first search
 *     with ef_construction on each of its layers, M neighbours per layer by
 *     the diversity heuristic (keep e unless a kept r has d(e, r) <
 *     d(node, e)); then reverse links grouped by target, in ascending
 *     source id, a full list (2M on layer 0, M above) re-selected by the
 *     same heuristic;
 *   - distances in FP32 in one order: element j summed by lane (j / 4) mod
 *     16 of 16 lanes in ascending j (L2 by fused multiply-add), the lanes
 *     combined pairwise (o = 8, 4, 2, 1).
 * The result is deterministic and, for metrics 1-3, identical to the CPU
 * input builder's (same steps, same distance order) for the same arguments.
 * metric_p is read for metric 4 only (in [0.2, 2]).
 * base: host, n x d FP32 row-major (copied; the context's loaded index is
 * not used or changed). *out receives a graph the caller frees with
 * uhnsw_built_graph_free.
 * Errors: EINVAL (NULL, n < 1, d outside [1, UHNSW_DMAX], metric or metric_p, M outside
 * [2, 31], ef_construction outside [1, UHNSW_EFMAX], batch_max outside
 * [1, 65536], a non-finite value), EUNSUPPORTED (upper layers above 2^31
 * ids), ENOMEM, EDEVICE; the message is uhnsw_last_error(ctx). */
#define UHNSW_METRIC_L1 1
#define UHNSW_METRIC_L2 2
#define UHNSW_METRIC_L05 3
#define UHNSW_METRIC_LP 4
typedef struct uhnsw_built_graph uhnsw_built_graph;
int uhnsw_build_graph(uhnsw_ctx *ctx, const float *base, int64_t n, int32_t d, int32_t metric, float metric_p,
                      int32_t M, int32_t ef_construction, uint64_t seed, int32_t batch_max,
                      uhnsw_built_graph **out);

/* The built graph as a uhnsw_graph (per-layer CSR; pointers into *g, valid
 * until uhnsw_built_graph_free), ready for uhnsw_index.graphs[]; the build's
 * wall time in seconds and its batch count (either may be NULL). */
int uhnsw_built_graph_view(const uhnsw_built_graph *g, uhnsw_graph *out, double *build_seconds,
                           int64_t *batches);
void uhnsw_built_graph_free(uhnsw_built_graph *g);

/* ------------------------------------------------------------ serving form
 * Continuous batching over the loaded index. Queries are admitted into
 * slots as they arrive; a dispatcher thread launches whatever is pending as
 * one fused walk+verify launch on the first idle stream, so batches that
 * arrive while others run overlap on the device. Admission: at most
 * max_inflight queries at once (default: the device's resident-wave
 * capacity for the fused kernel, one wave per query: CUs times the waves
 * per CU its LDS plan for k_max, ef_max and the visited-cache size and its
 * registers allow, from the occupancy query) and per-stream device buffers
 * within hbm_budget. A query's result is the same whichever batch carries
 * it. While a server runs, the context must not be used for other searches
 * and must not be destroyed. */
typedef struct uhnsw_server uhnsw_server;

typedef struct {
    int32_t k_max;            /* largest K a request may ask for (<= KMAX)   */
    int32_t ef_max;           /* largest ef (<= EFMAX)                        */
    int32_t max_inflight;     /* query slots, 0 = resident-wave capacity      */
    int32_t max_batch;        /* queries per launch, 0 = capacity / streams   */
    int32_t streams;          /* concurrent launches, 0 = 2 (<= 16)           */
    int32_t reserved;
    int64_t hbm_budget;       /* bytes for per-stream buffers, 0 = no limit  */
    uhnsw_params params;      /* Algorithm 1 parameters; launches are fused   */
} uhnsw_serve_config;

typedef struct {
    uint64_t tag;             /* the submitter's tag                          */
    int32_t status;           /* UHNSW_OK, UHNSW_EINVAL (bad query), EDEVICE  */
    int32_t nres;             /* valid entries in ids / dists                 */
    double submit_us;         /* host clock (us since server start): admitted */
    double launch_us;         /* its batch was launched                       */
    double done_us;           /* its batch was seen complete                  */
    uhnsw_stats stats;
    int64_t ids[UHNSW_KMAX];  /* ascending (d_p, id); -1 padded               */
    float dists[UHNSW_KMAX];  /* +inf padded                                  */
} uhnsw_serve_result;

void uhnsw_serve_default_config(uhnsw_serve_config *cfg);

/* Start a server on a context with a loaded index. Until uhnsw_serve_stop
 * the server's thread searches on the context: the caller makes no other
 * call on it, and uhnsw_load_graphs refuses with ESTATE.
 * Errors: EINVAL (limits), ESTATE (no index), ENOMEM, EBUSY (hbm_budget
 * below one query per stream). */
int uhnsw_serve_start(uhnsw_ctx *ctx, const uhnsw_serve_config *cfg, uhnsw_server **out);

/* Admit one query (copied; q has d floats). Thread-safe.
 * Errors: EINVAL (p outside the index's range, k, ef out of range or q not
 * finite), EBUSY (no free
 * slot: retry after polling), ESTATE (stopping), or a sticky device error. */
int uhnsw_serve_submit(uhnsw_server *srv, const float *q, float p, int32_t k, int32_t ef, uint64_t tag);

/* Take up to max finished results (any order). Thread-safe. */
int uhnsw_serve_poll(uhnsw_server *srv, uhnsw_serve_result *out, int32_t max, int32_t *n_out);

/* Counters: info[0] slots, [1] free slots, [2] pending, [3] batches
 * launched, [4] queries completed, [5] most batches in flight at once,
 * [6] batch size limit, [7] streams, [8] resident waves per CU of the
 * fused kernel under the LDS plan, [9] CUs. info has 10 entries. */
int uhnsw_serve_info(uhnsw_server *srv, int64_t *info);

/* Drive the server with a fixed arrival schedule (arrival_us[i] = offset of
 * arrival i from the call, ascending): submit each at its time (waiting for
 * slots when busy) and collect every result. Arrival i carries the query
 * vector queries[qidx[i]] (qidx may be NULL: queries[i]; the caller promises
 * qidx[i] indexes a row of queries) with p[i], k[i], ef[i]. ids / dists [n x out_k]
 * receive the first out_k entries of query i's row (-1 / +inf padded),
 * stats [n] its counters (may be NULL), times [n x 3] its scheduled arrival,
 * launch and completion in microseconds of the caller's clock (so
 * completion - arrival includes queueing), status [n] its status.
 * Synchronous. Errors: EINVAL (NULL array, out_k outside [1, KMAX]), or a
 * query's submit error. */
int uhnsw_serve_drive(uhnsw_server *srv, int64_t n, const float *queries, const int32_t *qidx, const float *p,
                      const int32_t *k, const int32_t *ef, const double *arrival_us, int32_t out_k, int64_t *ids,
                      float *dists, uhnsw_stats *stats, double *times, int32_t *status);

/* Finish in-flight work, stop the dispatcher, free the server. Returns the
 * server's sticky error (UHNSW_OK if its launches all succeeded); the
 * message of the last failure any serving call met is then what
 * uhnsw_last_error(ctx) returns. */
int uhnsw_serve_stop(uhnsw_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* UHNSW_H */
