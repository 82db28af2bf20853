// Internal structures shared by the host side and the kernels of libuhnsw.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "uhnsw.h"

namespace uhnsw {

constexpr int kWave = 64;
constexpr int kUCap = 64;            // neighbours gathered per walk step (beam_width * M0)
constexpr uint32_t kExpBit = 0x80000000u;
// Visited cache: 16-bit tags in sets of kVisWays (8). With 2^bits tags and
// ids below 2^kbits a tag needs kbits - bits + kVisWayBits bits, plus one for
// "empty", within 16.
constexpr int kVisWayBits = 3;
constexpr int kVisWays = 1 << kVisWayBits;
inline constexpr bool vis_tags_fit(int kbits, int bits) { return kbits - bits + kVisWayBits <= 15; }
constexpr uint32_t kIdMask = 0x7fffffffu;

// Row layout of one stored vector: element j is read by lane (j / V) % G of
// a G-lane group, in chunk j / (G * V); NCH chunks cover the padded row.
enum LayoutId : int { L8x4x1 = 0, L8x4x2, L8x4x4, L16x4x4, L32x4x4, L64x4x4, kNumLayouts };

struct LayoutInfo {
    int G, V, NCH;
};
inline LayoutInfo layout_info(int id) {
    static const LayoutInfo t[kNumLayouts] = {{8, 4, 1}, {8, 4, 2}, {8, 4, 4}, {16, 4, 4}, {32, 4, 4}, {64, 4, 4}};
    return t[id];
}
inline int layout_for_dim(int d) {
    if (d <= 32) return L8x4x1;
    if (d <= 64) return L8x4x2;
    if (d <= 128) return L8x4x4;
    if (d <= 256) return L16x4x4;
    if (d <= 512) return L32x4x4;
    return L64x4x4;
}

struct DevGraph {
    const int32_t *adj0;    // [n * M0], -1 padded
    const int32_t *up_off;  // [n], row in up_adj of the node's layer 1, -1 on level-0 nodes
    const int32_t *up_adj;  // [rows * M], -1 padded, valid ids first
    int32_t entry, max_level, M, M0;
};

struct SearchArgs {
    // index
    const void *walk_base;  // walk rows (storage type), pitch elements each
    const float *f32_base;  // FP32 rows for verification
    int64_t pitch;          // elements per row (both copies share it)
    int32_t n, d, storage;
    DevGraph g[2];
    // queries
    const float *queries;   // [nq x d]
    const float *p;
    const int32_t *k;
    const int32_t *ef;
    int64_t nq;
    int32_t k_max, ef_max;
    // Algorithm 1 parameters
    float cutoff;
    int32_t t_param, kappa_param, beam, early_abort;
    // m = ceil(tau * K) for K = 0 .. UHNSW_KMAX, capped at K + 1 (a count of
    // at most K never reaches it): passed by value, so every launch and every
    // captured graph carries its own tau's table
    uint16_t mtab[UHNSW_KMAX + 1];
    // LDS plan (per wave)
    int32_t ef_cap, vis_bits, vis_kbits, kv_cap, lds_wave_bytes, waves_per_block;
    // candidate lists (walk -> verify)
    int32_t *cand_ids;
    float *cand_keys;
    int32_t c_stride;
    int32_t *ncand;         // [nq]
    // outputs
    int64_t *ids;
    float *dists;
    int32_t k_stride;
    uhnsw_stats *stats;
    // persistent scheduling
    int32_t *counter;       // nullptr: one wave per query by grid position
    const int32_t *order;   // persistent order of queries (nullptr: 0..nq-1)
    // descent done by a pre-pass (nullptr: the walk descends itself)
    const int32_t *entry;   // [nq] layer-0 entry node
    const float *ekey;      // [nq] its base-metric key
    const int32_t *dnb;     // [nq] base distances the descent computed
    // index variant: 0 = G1 (L1) / G2 (L2), 1 = G_0.5 (L0.5) / G_1 (L1) and
    // the per-p variant (walk_p > 0); picks the kernel instantiation, read
    // on the host only
    int32_t ext;
    // every base value is 0 or at least 2^-72 in magnitude (the extended
    // walk may then take the short correctly rounded root)
    int32_t l05_fast;
    // every base value is an integer in [0, 255] (the extended walk may then
    // read its roots from a table)
    int32_t l05_table;
    // the per-p variant (ext = 1 kernels): graph 0 is walked under
    // sum |x - q|^walk_p; 0 for the other variants
    float walk_p;
    // the index variant's p range (queries outside are flagged UHNSW_QBAD)
    float p_lo, p_hi;
};

// Cost-ordered launch: a pre-pass descends every query and orders the
// queries by predicted walk length, largest first: the layer-0 entry
// distance relative to the mean of the query's graph (a far entry point
// predicts a long walk) times ef relative to the batch's mean ef (the walk
// expands at least ef entries). Starting the long walks first shortens the
// launch's tail.
constexpr int kOrderBuckets = 64;
struct OrderArgs {
    int32_t *entry;   // [nq] out: layer-0 entry node (-1: query not searchable)
    float *ekey;      // [nq] out: its key
    int32_t *dnb;     // [nq] out: base distances of the descent
    float *dist;      // [nq] out: entry distance in the graph's metric (L1, or L2)
    float *gsum;      // [6] out: (distance sum, count) per graph, then (ef sum, count)
    int32_t *bcnt;    // [2 * kOrderBuckets] bucket counts, then cursors; zeroed by the caller
    int32_t *order;   // [nq] out
};

// The fixed scratch region of the entry point that allocates nothing: its
// size, and its device address on `device` (looked up once per device).
constexpr size_t kNoAllocScratchBytes = (size_t)UHNSW_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, void **out);

// Launchers (uhnsw_kernels.hip). Return the HIP status of the launch.
hipError_t launch_walk(const SearchArgs &a, int layout, int grid, hipStream_t s);
hipError_t launch_verify(const SearchArgs &a, int layout, int grid, hipStream_t s);
hipError_t launch_search(const SearchArgs &a, int layout, int grid, hipStream_t s);
// descent pre-pass + ordering for the cost-ordered launch; `a` as for the walk
hipError_t launch_order(const SearchArgs &a, const OrderArgs &o, int layout, hipStream_t s);
hipError_t launch_fill_i32(int32_t *dst, int32_t v, int64_t n, hipStream_t s);
// ceiling probes (measurement only): `blocks` x 4 waves; a gather wave reads
// iters x 32 random rows of row_bytes (128, 256 or 512) from rows of `pitch`
// floats; a transcendental thread runs iters x 8 exp/log pairs
hipError_t launch_gather_probe(const float *base, int64_t n, int64_t pitch, int row_bytes, int blocks, int iters,
                               uint32_t seed, float *sink, hipStream_t s);
hipError_t launch_trans_probe(int blocks, int iters, float *sink, hipStream_t s);
hipError_t launch_convert(const float *src, void *dst, int64_t count, int storage, hipStream_t s);
int walk_lds_bytes(int ef_cap, int vis_bits, int vis_kbits, bool ext);
int verify_lds_bytes(int kv_cap);
const void *walk_kernel_ptr(int layout, int storage, bool ext);
const void *verify_kernel_ptr(int layout);
const void *search_kernel_ptr(int layout, int storage, int beam, bool ext);
int ctx_dim(const uhnsw_ctx *c);
int ctx_variant(const uhnsw_ctx *c);
void ctx_servers(uhnsw_ctx *c, int delta);  // servers running on the context
bool p_in_range(int variant, float p);  // the index variant's p range
int ctx_device(const uhnsw_ctx *c);
void ctx_set_error(uhnsw_ctx *c, const char *msg);  // the message uhnsw_last_error returns
// resident waves per CU of the fused kernel under this LDS plan (occupancy)
int ctx_resident_waves(uhnsw_ctx *c, int k_max, int ef_max, const uhnsw_params *prm, int *waves_per_cu);

}  // namespace uhnsw
