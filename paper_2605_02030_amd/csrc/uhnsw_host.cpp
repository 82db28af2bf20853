// Host side of libuhnsw: context, validation, upload of the index to the
// device layout, and launch planning for the walk and verify kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "uhnsw.h"
#include "uhnsw_guard.h"
#include "uhnsw_internal.h"

using namespace uhnsw;

namespace {

thread_local std::string g_create_error;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void reset() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t want) {
        if (want <= bytes && p) return hipSuccess;
        reset();
        hipError_t e = hipMalloc(&p, want ? want : 1);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    template <typename T>
    T *as() const {
        return reinterpret_cast<T *>(p);
    }
};

// streams one context serves at once (each holds its own search scratch)
constexpr int kMaxStreams = 64;

// What a captured launch sequence depends on besides the kernels: the
// caller's pointers and sizes, the knobs, and `gen`, the context's scratch
// generation (bumped whenever a scratch buffer the kernels may address is
// reallocated), so a graph that baked in freed scratch is never replayed.
struct GraphKey {
    const void *ptrs[16];
    int64_t nq;
    int32_t ints[4];
    uhnsw_params prm;
    uint64_t gen;
};

struct GraphDev {
    DevBuf adj0, up_off, up_adj;
    int32_t entry = 0, max_level = 0, M = 0, M0 = 0;
};

}  // namespace

struct uhnsw_ctx {
    int device = 0;
    int num_cus = 0;
    void *noalloc = nullptr;  // the device's fixed scratch region (noalloc_scratch)
    hipStream_t stream = nullptr;
    bool loaded = false;
    bool failed = false;
    std::string err;
    // index
    int64_t n = 0;
    int32_t d = 0, storage = 0, layout = 0;
    int32_t variant = UHNSW_VARIANT_STD;
    float graph_p = 0.0f;  // UHNSW_VARIANT_PGRAPH
    std::atomic<int> servers{0};  // uhnsw_serve_start .. uhnsw_serve_stop
    bool l05_fast = false;   // every base value 0 or of magnitude >= 2^-72
    bool l05_table = false;  // every base value an integer in [0, 255]
    int64_t pitch = 0;
    DevBuf f32_base, walk_base;
    GraphDev g[2];
    uint64_t scratch_gen = 0;  // bumped on every scratch reallocation (GraphKey)
    // Per-launch-stream scratch: searches on different streams may run
    // concurrently, so everything a search writes besides the caller's
    // outputs (candidate lists, counts, default stats, the work counter,
    // timing events, the captured hipGraph) belongs to its stream.
    struct StreamSet {
        hipStream_t stream = nullptr;
        DevBuf cand_ids, cand_keys, ncand, stats, counter;
        DevBuf o_entry, o_ekey, o_dnb, o_dist, o_misc, o_order;  // cost-ordered launch
        // timing events: [0] start, [3] after the pre-pass, [1] after the
        // walk (or fused) kernel, [2] after verification
        hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
        bool timed = false;
        bool split = false;  // ev[3] recorded (not a graph replay)
        hipGraphExec_t gexec = nullptr;
        GraphKey gkey{};
    };
    std::vector<std::unique_ptr<StreamSet>> sets;
    StreamSet *last_set = nullptr;  // the most recent search
    // staging for the host-pointer entry point
    DevBuf s_q, s_p, s_k, s_ef, s_ids, s_dists, s_stats;
    hipStream_t cap_stream = nullptr;   // capture stream for hipGraphs
    hipStream_t tune_stream = nullptr;  // second stream of the pipelined autotuner
    int64_t graph_captures = 0;
    // host-pointer path under a hipGraph: pinned staging + the captured
    // sequence H2D copies -> kernels -> D2H copies
    struct Pinned {
        void *p = nullptr;
        size_t bytes = 0;
    } hp[7];
    hipGraphExec_t hgexec = nullptr;
    GraphKey hgkey{};
    // resident blocks per CU by (kernel, block size, LDS bytes), queried once
    // (also keeps the query out of any hipGraph capture)
    struct Occ {
        const void *kernel;
        int block;
        size_t lds;
        int per_cu;
    };
    std::vector<Occ> occ;
    // autotuner results keyed by (n, d, storage, ef bucket, k_max, beam, fused)
    std::vector<std::pair<uint64_t, uhnsw_params>> tuned;
};

namespace uhnsw {
// the p range of an index variant
void p_range(int variant, float *lo, float *hi) {
    *lo = variant == UHNSW_VARIANT_STD ? 0.5f : 0.2f;
    *hi = variant == UHNSW_VARIANT_EXT ? 1.0f : 2.0f;
}
bool p_in_range(int variant, float p) {
    float lo, hi;
    p_range(variant, &lo, &hi);
    return p >= lo && p <= hi;
}
int ctx_variant(const uhnsw_ctx *c) { return c->variant; }
void ctx_servers(uhnsw_ctx *c, int delta) { c->servers += delta; }
int ctx_dim(const uhnsw_ctx *c) { return c->d; }
int ctx_device(const uhnsw_ctx *c) { return c->device; }
void ctx_set_error(uhnsw_ctx *c, const char *msg) { c->err = msg; }
}  // namespace uhnsw

namespace {

int vfail(std::string *err, int code, const char *fmt, va_list ap) {
    char buf[512];
    vsnprintf(buf, sizeof buf, fmt, ap);
    *err = buf;
    return code;
}

int fail(uhnsw_ctx *c, int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfail(&c->err, code, fmt, ap);
    va_end(ap);
    return code;
}

// The same for checks that run without a context (the message goes to *err).
int fail(std::string *err, int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfail(err, code, fmt, ap);
    va_end(ap);
    return code;
}

int dev_fail(uhnsw_ctx *c, hipError_t e, const char *what) {
    c->failed = true;
    return fail(c, e == hipErrorOutOfMemory ? UHNSW_ENOMEM : UHNSW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_OR_FAIL(ctx, call)                             \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return dev_fail(ctx, e_, #call); \
    } while (0)

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Validate one graph against n and the node levels; returns 0 or EINVAL.
int check_graph(std::string *c, const uhnsw_graph &g, int64_t n, int which) {
    const char *nm = which == 0 ? "G1" : "G2";
    if (g.M < 1 || 2 * g.M > kWave) return fail(c, UHNSW_EINVAL, "%s: M=%d outside [1, 32]", nm, g.M);
    if (g.max_level < 0 || g.max_level >= UHNSW_MAX_LAYERS)
        return fail(c, UHNSW_EINVAL, "%s: max_level=%d outside [0, %d)", nm, g.max_level, UHNSW_MAX_LAYERS);
    if (!g.level || !g.row_ptr[0] || (!g.col[0] && n > 0))
        return fail(c, UHNSW_EINVAL, "%s: NULL level/row_ptr/col", nm);
    if (g.entry_point < 0 || g.entry_point >= n) return fail(c, UHNSW_EINVAL, "%s: entry point out of range", nm);
    int top = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (g.level[v] < 0 || g.level[v] >= UHNSW_MAX_LAYERS)
            return fail(c, UHNSW_EINVAL, "%s: level[%lld] out of range", nm, (long long)v);
        top = std::max<int>(top, g.level[v]);
    }
    if (top != g.max_level || g.level[g.entry_point] != g.max_level)
        return fail(c, UHNSW_EINVAL, "%s: entry point is not on the top layer %d", nm, g.max_level);
    for (int l = 0; l <= g.max_level; ++l) {
        const int64_t *rp = g.row_ptr[l];
        const int32_t *col = g.col[l];
        const int64_t rows = l == 0 ? n : g.n_nodes[l];
        const int deg_max = l == 0 ? 2 * g.M : g.M;
        if (!rp || (l > 0 && !g.nodes[l])) return fail(c, UHNSW_EINVAL, "%s: layer %d arrays missing", nm, l);
        int64_t on_layer = 0;
        for (int64_t v = 0; v < n; ++v) on_layer += g.level[v] >= l;
        if (rows != on_layer)
            return fail(c, UHNSW_EINVAL, "%s: layer %d lists %lld nodes, levels say %lld", nm, l, (long long)rows,
                        (long long)on_layer);
        if (rp[0] != 0) return fail(c, UHNSW_EINVAL, "%s: layer %d row_ptr[0] != 0", nm, l);
        for (int64_t r = 0; l > 0 && r < rows; ++r) {
            const int32_t v = g.nodes[l][r];
            if (v < 0 || v >= n || g.level[v] < l || (r > 0 && g.nodes[l][r - 1] >= v))
                return fail(c, UHNSW_EINVAL, "%s: layer %d nodes not ascending ids on the layer", nm, l);
        }
        for (int64_t r = 0; r < rows; ++r) {
            const int64_t deg = rp[r + 1] - rp[r];
            if (deg < 0 || deg > deg_max)
                return fail(c, UHNSW_EINVAL, "%s: layer %d row %lld degree %lld outside [0, %d]", nm, l,
                            (long long)r, (long long)deg, deg_max);
            const int32_t self = l == 0 ? (int32_t)r : g.nodes[l][r];
            int32_t row[kWave];
            for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
                const int32_t u = col[e];
                if (u < 0 || u >= n || g.level[u] < l)
                    return fail(c, UHNSW_EINVAL, "%s: layer %d edge to %d not on the layer", nm, l, u);
                if (u == self)
                    return fail(c, UHNSW_EINVAL, "%s: layer %d node %d lists itself as a neighbour", nm, l, u);
                row[e - rp[r]] = u;
            }
            // An HNSW neighbour list is a set (Sec. 2.2): the walk marks a
            // neighbour visited only after all of a row's ids were tested,
            // so an id listed twice would enter the candidate list twice.
            std::sort(row, row + deg);
            for (int64_t e = 1; e < deg; ++e)
                if (row[e] == row[e - 1])
                    return fail(c, UHNSW_EINVAL, "%s: layer %d node %d lists neighbour %d twice", nm, l, self,
                                row[e]);
        }
    }
    return UHNSW_OK;
}

int upload_graph(uhnsw_ctx *c, const uhnsw_graph &g, int64_t n, GraphDev &gd) {
    const int M = g.M, M0 = 2 * g.M;
    std::vector<int32_t> adj0((size_t)n * M0, -1);
    for (int64_t v = 0; v < n; ++v) {
        const int64_t b = g.row_ptr[0][v], e = g.row_ptr[0][v + 1];
        for (int64_t i = b; i < e; ++i) adj0[(size_t)v * M0 + (i - b)] = g.col[0][i];
    }
    std::vector<int32_t> up_off((size_t)n, -1);
    int64_t rows = 0;
    for (int64_t v = 0; v < n; ++v)
        if (g.level[v] > 0) {
            up_off[v] = (int32_t)rows;
            rows += g.level[v];
        }
    if (rows >= (int64_t)INT32_MAX / std::max(M, 1)) return fail(c, UHNSW_EINVAL, "upper layers too large");
    std::vector<int32_t> up_adj((size_t)std::max<int64_t>(rows, 1) * M, -1);
    for (int l = 1; l <= g.max_level; ++l) {
        for (int64_t r = 0; r < g.n_nodes[l]; ++r) {
            const int32_t v = g.nodes[l][r];
            const int64_t row = up_off[v] + (l - 1);
            const int64_t b = g.row_ptr[l][r], e = g.row_ptr[l][r + 1];
            for (int64_t i = b; i < e; ++i) up_adj[(size_t)row * M + (i - b)] = g.col[l][i];
        }
    }
    HIP_OR_FAIL(c, gd.adj0.ensure(adj0.size() * 4));
    HIP_OR_FAIL(c, gd.up_off.ensure(up_off.size() * 4));
    HIP_OR_FAIL(c, gd.up_adj.ensure(up_adj.size() * 4));
    HIP_OR_FAIL(c, hipMemcpy(gd.adj0.p, adj0.data(), adj0.size() * 4, hipMemcpyHostToDevice));
    HIP_OR_FAIL(c, hipMemcpy(gd.up_off.p, up_off.data(), up_off.size() * 4, hipMemcpyHostToDevice));
    HIP_OR_FAIL(c, hipMemcpy(gd.up_adj.p, up_adj.data(), up_adj.size() * 4, hipMemcpyHostToDevice));
    gd.entry = g.entry_point;
    gd.max_level = g.max_level;
    gd.M = M;
    gd.M0 = M0;
    return UHNSW_OK;
}

struct Plan {
    int ef_cap, vis_bits, vis_kbits, kv_cap, wpb, walk_bytes, verify_bytes, search_bytes;
};

int make_plan(uhnsw_ctx *c, int k_max, int ef_max, const uhnsw_params &prm, Plan *pl) {
    pl->ef_cap = round_up(std::max(ef_max, 1), 4);
    // cache geometry for a slot count: log2 slots, and the key width when
    // 16-bit quotient slots suffice for the id range (see VisCache), else 0
    auto vis_geometry = [c](int slots, int *bits, int *kbits) {
        int b = 0;
        while ((1 << b) < slots) ++b;
        int kb = 1;
        while (kb < 31 && ((int64_t)1 << kb) < c->n) ++kb;
        if (kb < b + 1) kb = b + 1;
        *bits = b;
        *kbits = vis_tags_fit(kb, b) ? kb : 0;
    };
    int slots = prm.visited_slots;
    if (slots <= 0 && ef_max > 512) {
        slots = 8192;
    } else if (slots <= 0) {
        // The largest cache that keeps a wave's LDS within 11 KiB (14 waves
        // per CU). A larger cache forgets fewer nodes (fewer repeated
        // distances), a smaller one leaves room for more waves; measured on
        // the 1M x 128 workload: at ef 256, 4,096 slots (10.5 KiB) beat
        // 2,048 by 4 %; at ef 384 and 512, 4,096 slots would leave 12-13
        // waves per CU and 2,048 wins by 16 % and 41 %.
        constexpr int kLdsWaveBudget = 11 * 1024;
        for (slots = 8192; slots > 1024; slots /= 2) {
            int b, kb;
            vis_geometry(slots, &b, &kb);
            if (walk_lds_bytes(pl->ef_cap, b, kb, c->variant == UHNSW_VARIANT_EXT) <= kLdsWaveBudget) break;
        }
    }
    int bits = 0, kbits = 0;
    vis_geometry(slots, &bits, &kbits);
    if (bits < 6 || bits > 14) return fail(c, UHNSW_EINVAL, "visited_slots %d outside [64, 16384]", slots);
    pl->vis_bits = bits;
    pl->vis_kbits = kbits;
    const int kappa_max = prm.kappa > 0 ? prm.kappa : std::max(k_max, 2);
    pl->kv_cap = round_up(std::max(k_max, kappa_max), 4);
    pl->walk_bytes = walk_lds_bytes(pl->ef_cap, pl->vis_bits, pl->vis_kbits, c->variant == UHNSW_VARIANT_EXT);
    pl->verify_bytes = verify_lds_bytes(pl->kv_cap);
    // fused kernel: the verification's arrays follow the walk's list W
    pl->search_bytes = std::max(pl->walk_bytes, pl->ef_cap * 8 + pl->verify_bytes);
    const int per_wave = prm.fused ? pl->search_bytes : std::max(pl->walk_bytes, pl->verify_bytes);
    // one wave per block by default: LDS is granted per block, and single-
    // wave blocks pack a CU's 160 KiB without leftovers (at 10.5 KiB per
    // wave, four-wave blocks fit 3 per CU, 12 waves; one-wave blocks 15)
    pl->wpb = prm.waves_per_block > 0 ? prm.waves_per_block : 1;
    if (pl->wpb > 4) return fail(c, UHNSW_EINVAL, "waves_per_block %d > 4", pl->wpb);
    if ((size_t)per_wave * pl->wpb > 64 * 1024)
        return fail(c, UHNSW_EUNSUPPORTED, "LDS plan %d B/wave x %d waves exceeds 64 KiB per block", per_wave,
                    pl->wpb);
    return UHNSW_OK;
}

// Algorithm 1's stop test |R_new n R| / K >= tau as the integer test
// |R_new n R| >= m, m = ceil(tau K) (the 1e-9 guard keeps 0.92 * 100 at 92);
// m above K never fires, so it is capped at K + 1.
void fill_mtab(double tau, uint16_t *tab) {
    tab[0] = 0;
    for (int K = 1; K <= UHNSW_KMAX; ++K) {
        const double m = std::ceil(tau * (double)K - 1e-9);
        tab[K] = (uint16_t)(m > K ? K + 1 : (m < 0 ? 0 : m));
    }
}

// Scratch that the kernels address: a reallocation moves it, so every
// captured graph that may hold the old address is invalidated.
hipError_t ensure_scratch(uhnsw_ctx *c, DevBuf &b, size_t want) {
    void *old = b.p;
    const size_t old_bytes = b.bytes;
    hipError_t e = b.ensure(want);
    if (b.p != old || b.bytes != old_bytes) ++c->scratch_gen;
    return e;
}

int check_params(uhnsw_ctx *c, const uhnsw_params &prm) {
    if (!(prm.tau > 0.0) || !std::isfinite(prm.tau)) return fail(c, UHNSW_EINVAL, "tau must be positive");
    if (!std::isfinite(prm.cutoff) || prm.cutoff < 0.0f)
        return fail(c, UHNSW_EINVAL, "cutoff must be finite and >= 0 (0: the index's default)");
    if (prm.t < 0 || prm.kappa < 0) return fail(c, UHNSW_EINVAL, "t and kappa must be >= 0");
    if (prm.beam_width < 1 || prm.beam_width > 2) return fail(c, UHNSW_EINVAL, "beam_width must be 1 or 2");
    if (prm.persistent < 0 || prm.persistent > 3) return fail(c, UHNSW_EINVAL, "persistent must be 0 .. 3");
    for (int i = 0; i < 2; ++i)
        if (prm.beam_width * c->g[i].M0 > kUCap)
            return fail(c, UHNSW_EINVAL, "beam_width %d x 2M = %d exceeds %d lanes", prm.beam_width,
                        prm.beam_width * c->g[i].M0, kUCap);
    return UHNSW_OK;
}

}  // namespace

namespace {

// Whole-file reader with bounds-checked takes (little-endian host).
struct FileBuf {
    std::vector<char> b;
    size_t at = 0;
    bool ok = true;
    template <typename T>
    T take() {
        T v{};
        if (at + sizeof(T) > b.size()) {
            ok = false;
            return v;
        }
        std::memcpy(&v, b.data() + at, sizeof(T));
        at += sizeof(T);
        return v;
    }
    template <typename T>
    bool copy(int64_t count, std::vector<T> *out) {  // into aligned storage (the file may not be)
        if (count < 0 || at + (size_t)count * sizeof(T) > b.size()) {
            ok = false;
            return false;
        }
        out->resize((size_t)count);
        if (count) std::memcpy(out->data(), b.data() + at, (size_t)count * sizeof(T));
        at += (size_t)count * sizeof(T);
        return true;
    }
};

bool read_file(const char *path, FileBuf *f) {
    FILE *fp = path ? std::fopen(path, "rb") : nullptr;
    if (!fp) return false;
    bool good = std::fseek(fp, 0, SEEK_END) == 0;
    const long size = good ? std::ftell(fp) : -1;
    good = good && size >= 0 && std::fseek(fp, 0, SEEK_SET) == 0;
    if (good) {
        f->b.resize((size_t)size);
        good = size == 0 || std::fread(f->b.data(), 1, (size_t)size, fp) == (size_t)size;
    }
    std::fclose(fp);
    return good;
}

// Parsed graph file: owns aligned copies of every array uhnsw_graph points to.
struct GraphFile {
    int32_t n = 0;
    uhnsw_graph g{};
    std::vector<int8_t> level;
    std::vector<std::vector<int64_t>> row_ptr;
    std::vector<std::vector<int32_t>> col, nodes;
};

int parse_graph(std::string *c, const char *path, GraphFile *out) {
    FileBuf f;
    if (!read_file(path, &f)) return fail(c, UHNSW_EIO, "cannot read %s", path ? path : "(null)");
    std::vector<char> magic;
    if (!f.copy(4, &magic) || std::memcmp(magic.data(), "UHG1", 4) != 0)
        return fail(c, UHNSW_EIO, "%s: not a UHG1 graph file", path);
    const int32_t n = f.take<int32_t>(), M = f.take<int32_t>(), ml = f.take<int32_t>(), ep = f.take<int32_t>();
    if (!f.ok || n < 1 || ml < 0 || ml >= UHNSW_MAX_LAYERS)
        return fail(c, UHNSW_EIO, "%s: bad header (n=%d, max_level=%d)", path, n, ml);
    if (!f.copy(n, &out->level)) return fail(c, UHNSW_EIO, "%s: short file (levels)", path);
    out->n = n;
    out->row_ptr.resize(ml + 1);
    out->col.resize(ml + 1);
    out->nodes.resize(ml + 1);
    out->g.M = M;
    out->g.max_level = ml;
    out->g.entry_point = ep;
    out->g.level = out->level.data();
    for (int l = 0; l <= ml; ++l) {
        const int64_t nl = f.take<int64_t>();
        if (!f.ok || nl < 0 || nl > n || (l == 0 && nl != n)) return fail(c, UHNSW_EIO, "%s: bad layer %d size", path, l);
        if (!f.copy(nl + 1, &out->row_ptr[l])) return fail(c, UHNSW_EIO, "%s: short file (layer %d rows)", path, l);
        const int64_t ne = out->row_ptr[l][nl];
        if (ne < 0 || ne > (int64_t)64 * n) return fail(c, UHNSW_EIO, "%s: bad edge count on layer %d", path, l);
        if (!f.copy(ne, &out->col[l])) return fail(c, UHNSW_EIO, "%s: short file (layer %d edges)", path, l);
        if (out->col[l].empty()) out->col[l].push_back(0);  // a valid pointer for empty layers
        if (l >= 1) {
            if (!f.copy(nl, &out->nodes[l])) return fail(c, UHNSW_EIO, "%s: short file (layer %d nodes)", path, l);
            if (out->nodes[l].empty()) out->nodes[l].push_back(0);
            out->g.nodes[l] = out->nodes[l].data();
        }
        out->g.n_nodes[l] = nl;
        out->g.row_ptr[l] = out->row_ptr[l].data();
        out->g.col[l] = out->col[l].data();
    }
    return UHNSW_OK;
}

// Everything uhnsw_load_graphs checks before it touches the device.
int check_index(std::string *err, const uhnsw_index *idx) {
    if (!idx || !idx->base) return fail(err, UHNSW_EINVAL, "index or base is NULL");
    if (idx->n < 1 || idx->n > INT32_MAX) return fail(err, UHNSW_EINVAL, "n=%lld outside [1, 2^31)", (long long)idx->n);
    if (idx->d < 1 || idx->d > UHNSW_DMAX) return fail(err, UHNSW_EINVAL, "d=%d outside [1, %d]", idx->d, UHNSW_DMAX);
    if (idx->storage < UHNSW_STORE_F32 || idx->storage > UHNSW_STORE_F16)
        return fail(err, UHNSW_EINVAL, "unknown storage %d", idx->storage);
    if (idx->variant != UHNSW_VARIANT_STD && idx->variant != UHNSW_VARIANT_EXT &&
        idx->variant != UHNSW_VARIANT_PGRAPH)
        return fail(err, UHNSW_EINVAL, "unknown variant %d", idx->variant);
    if (idx->variant == UHNSW_VARIANT_PGRAPH && !(idx->graph_p >= 0.2f && idx->graph_p <= 2.0f))
        return fail(err, UHNSW_EINVAL, "graph_p=%g outside [0.2, 2]", (double)idx->graph_p);
    for (int i = 0; i < 2; ++i) {
        int r = check_graph(err, idx->graphs[i], idx->n, i);
        if (r) return r;
    }
    for (int64_t i = 0; i < idx->n * idx->d; ++i)
        if (!std::isfinite(idx->base[i]))
            return fail(err, UHNSW_EINVAL, "base value %lld is not finite", (long long)i);
    return UHNSW_OK;
}

// The three index files, parsed into an index whose arrays this object owns.
struct IndexFiles {
    std::vector<float> base;
    GraphFile g1, g2;
    uhnsw_index idx{};
};

int read_index_files(std::string *err, const char *vec_path, const char *g1_path, const char *g2_path,
                     int32_t storage, int32_t variant, IndexFiles *out) {
    FileBuf vf;
    if (!read_file(vec_path, &vf)) return fail(err, UHNSW_EIO, "cannot read %s", vec_path ? vec_path : "(null)");
    const int32_t n = vf.take<int32_t>(), d = vf.take<int32_t>();
    if (!vf.ok || n < 1 || d < 1 || d > UHNSW_DMAX)
        return fail(err, UHNSW_EIO, "%s: bad header (n=%d, d=%d)", vec_path, n, d);
    if (!vf.copy((int64_t)n * d, &out->base)) return fail(err, UHNSW_EIO, "%s: short file", vec_path);
    vf.b.clear();
    int r = parse_graph(err, g1_path, &out->g1);
    if (r) return r;
    if ((r = parse_graph(err, g2_path, &out->g2))) return r;
    if (out->g1.n != n || out->g2.n != n)
        return fail(err, UHNSW_EIO, "graph files hold %d / %d nodes, vectors %d", out->g1.n, out->g2.n, n);
    out->idx.n = n;
    out->idx.d = d;
    out->idx.base = out->base.data();
    out->idx.storage = storage;
    out->idx.variant = variant;
    out->idx.graphs[0] = out->g1.g;
    out->idx.graphs[1] = out->g2.g;
    return UHNSW_OK;
}

int check_result(const std::string &err, int r, char *msg, int32_t msg_len) {
    if (msg && msg_len > 0) std::snprintf(msg, (size_t)msg_len, "%s", r ? err.c_str() : "");
    return r;
}

}  // namespace

namespace uhnsw {
// Waves of the fused kernel that stay resident per CU for this index and
// these limits: its LDS plan (the list W, the visited cache, merge and
// verification scratch per wave) and registers, as the occupancy query
// reports them.
int ctx_resident_waves(uhnsw_ctx *c, int k_max, int ef_max, const uhnsw_params *prm_in, int *waves_per_cu) {
    if (!c->loaded) return fail(c, UHNSW_ESTATE, "no index loaded");
    uhnsw_params prm = *prm_in;
    prm.fused = 1;
    int r = check_params(c, prm);
    if (r) return r;
    Plan pl;
    if ((r = make_plan(c, k_max, ef_max, prm, &pl))) return r;
    const void *kp = search_kernel_ptr(c->layout, c->storage, prm.beam_width, c->variant == UHNSW_VARIANT_EXT);
    int blocks = 0;
    HIP_OR_FAIL(c, hipSetDevice(c->device));
    HIP_OR_FAIL(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kp, pl.wpb * kWave,
                                                                 (size_t)pl.search_bytes * pl.wpb));
    *waves_per_cu = blocks * pl.wpb;
    return UHNSW_OK;
}
}  // namespace uhnsw

// ================================================================ C ABI
extern "C" {

void uhnsw_default_params(uhnsw_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->tau = 0.92;
    p->cutoff = 0.0f;  // the index's default: 1.4, or 0.6 for the extended pair
    p->beam_width = 1;
    p->early_abort = 1;
    p->persistent = 3;  // cost-ordered launch: same results, shorter tail
}

static int create_body(int device, uhnsw_ctx **out) {
    if (!out) {
        g_create_error = "out is NULL";
        return UHNSW_EINVAL;
    }
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || device < 0 || device >= ndev) {
        g_create_error = "no HIP device " + std::to_string(device) + " (" +
                         (e != hipSuccess ? hipGetErrorString(e) : std::to_string(ndev) + " present") + ")";
        return e != hipSuccess ? UHNSW_EDEVICE : UHNSW_EINVAL;
    }
    uhnsw_ctx *c = new (std::nothrow) uhnsw_ctx();
    if (!c) {
        g_create_error = "out of host memory";
        return UHNSW_ENOMEM;
    }
    c->device = device;
    if ((e = hipSetDevice(device)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = noalloc_scratch(device, &c->noalloc)) != hipSuccess) {
        g_create_error = std::string("device setup: ") + hipGetErrorString(e);
        if (c->stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return UHNSW_EDEVICE;
    }
    *out = c;
    return UHNSW_OK;
}

int uhnsw_create(int device, uhnsw_ctx **out) {
    const auto body = [&] { return create_body(device, out); };
    return no_throw("uhnsw_create", body, [&](const char *w) { g_create_error = w; });
}

void uhnsw_destroy(uhnsw_ctx *c) {
    if (!c) return;
    if (c->servers.load() > 0) {  // a server's thread still searches on it: keep it alive
        c->err = "uhnsw_destroy refused: a server is running on this context";
        return;
    }
    (void)hipSetDevice(c->device);
    // Wait for every search of this context: the caller's streams may already
    // be gone, so the device is synchronised rather than each stream.
    (void)hipDeviceSynchronize();
    for (auto &S : c->sets) {
        for (auto &ev : S->ev)
            if (ev) (void)hipEventDestroy(ev);
        DevBuf *sb[] = {&S->cand_ids, &S->cand_keys, &S->ncand, &S->stats, &S->counter, &S->o_entry,
                        &S->o_ekey, &S->o_dnb, &S->o_dist, &S->o_misc, &S->o_order};
        for (DevBuf *b : sb) b->reset();
        if (S->gexec) (void)hipGraphExecDestroy(S->gexec);
    }
    c->sets.clear();
    DevBuf *bufs[] = {&c->f32_base, &c->walk_base, &c->s_q, &c->s_p, &c->s_k, &c->s_ef, &c->s_ids,
                      &c->s_dists, &c->s_stats};
    for (DevBuf *b : bufs) b->reset();
    for (auto &g : c->g) {
        g.adj0.reset();
        g.up_off.reset();
        g.up_adj.reset();
    }
    if (c->hgexec) (void)hipGraphExecDestroy(c->hgexec);
    for (auto &h : c->hp)
        if (h.p) (void)hipHostFree(h.p);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->tune_stream) (void)hipStreamDestroy(c->tune_stream);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *uhnsw_last_error(const uhnsw_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

static int reset_body(uhnsw_ctx *c) {
    if (!c) return UHNSW_EINVAL;
    if (c->servers.load() > 0) return fail(c, UHNSW_ESTATE, "uhnsw_reset refused: a server is running");
    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipGetLastError();  // clear a non-sticky error left by the failure
    if (e != hipSuccess) {
        c->failed = true;
        return fail(c, UHNSW_EDEVICE, "uhnsw_reset: the device still reports %s; destroy the context",
                    hipGetErrorString(e));
    }
    // Everything a failed call may have left half made: captured graphs and
    // the per-stream and staging scratch (reallocated on next use).
    for (auto &S : c->sets) {
        if (S->gexec) (void)hipGraphExecDestroy(S->gexec);
        S->gexec = nullptr;
        S->gkey = GraphKey{};
        DevBuf *sb[] = {&S->cand_ids, &S->cand_keys, &S->ncand, &S->stats, &S->counter, &S->o_entry,
                        &S->o_ekey, &S->o_dnb, &S->o_dist, &S->o_misc, &S->o_order};
        for (DevBuf *b : sb) b->reset();
    }
    if (c->hgexec) (void)hipGraphExecDestroy(c->hgexec);
    c->hgexec = nullptr;
    c->hgkey = GraphKey{};
    DevBuf *bufs[] = {&c->s_q, &c->s_p, &c->s_k, &c->s_ef, &c->s_ids, &c->s_dists, &c->s_stats};
    for (DevBuf *b : bufs) b->reset();
    ++c->scratch_gen;
    c->failed = false;
    c->err.clear();
    return UHNSW_OK;
}

int uhnsw_reset(uhnsw_ctx *c) {
    const auto body = [&] { return reset_body(c); };
    return no_throw("uhnsw_reset", body, [&](const char *w) { if (c) ctx_set_error(c, w); });
}

static int load_graphs_body(uhnsw_ctx *c, const uhnsw_index *idx) {
    if (!c) return UHNSW_EINVAL;
    int r0 = check_index(&c->err, idx);
    if (r0) return r0;
    if (c->servers.load() > 0) return fail(c, UHNSW_ESTATE, "a server is running on this context");
    HIP_OR_FAIL(c, hipSetDevice(c->device));
    // Searches still in flight read the buffers about to be replaced, and
    // captured launch graphs hold the old index's pointers, sizes and kernel
    // variant as baked arguments: wait for the device, then drop the graphs
    // so the next graph search captures afresh.
    HIP_OR_FAIL(c, hipDeviceSynchronize());
    for (auto &S : c->sets)
        if (S->gexec) {
            (void)hipGraphExecDestroy(S->gexec);
            S->gexec = nullptr;
            S->gkey = GraphKey{};
        }
    if (c->hgexec) {
        (void)hipGraphExecDestroy(c->hgexec);
        c->hgexec = nullptr;
        c->hgkey = GraphKey{};
    }
    c->loaded = false;
    const int layout = layout_for_dim(idx->d);
    const LayoutInfo li = layout_info(layout);
    const int64_t pitch = (int64_t)li.G * li.V * li.NCH;
    const int64_t n = idx->n;
    {
        std::vector<float> rows((size_t)n * pitch, 0.0f);
        for (int64_t v = 0; v < n; ++v)
            std::memcpy(&rows[(size_t)v * pitch], idx->base + (size_t)v * idx->d, sizeof(float) * idx->d);
        HIP_OR_FAIL(c, c->f32_base.ensure(rows.size() * 4));
        HIP_OR_FAIL(c, hipMemcpy(c->f32_base.p, rows.data(), rows.size() * 4, hipMemcpyHostToDevice));
    }
    if (idx->storage != UHNSW_STORE_F32) {
        HIP_OR_FAIL(c, c->walk_base.ensure((size_t)n * pitch * 2));
        HIP_OR_FAIL(c, launch_convert(c->f32_base.as<float>(), c->walk_base.p, n * pitch, idx->storage, c->stream));
        HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    } else {
        c->walk_base.reset();
    }
    for (int i = 0; i < 2; ++i) {
        int r = upload_graph(c, idx->graphs[i], n, c->g[i]);
        if (r) return r;
    }
    c->n = n;
    c->d = idx->d;
    c->storage = idx->storage;
    c->variant = idx->variant;
    c->graph_p = idx->variant == UHNSW_VARIANT_PGRAPH ? idx->graph_p : 0.0f;
    c->l05_fast = c->l05_table = true;
    for (int64_t i = 0; i < n * idx->d && (c->l05_fast || c->l05_table); ++i) {
        const float v = idx->base[i];
        c->l05_fast = c->l05_fast && (v == 0.0f || std::fabs(v) >= 0x1p-72f);
        c->l05_table = c->l05_table && v >= 0.0f && v <= 255.0f && v == std::rint(v);
    }
    c->layout = layout;
    c->pitch = pitch;
    c->loaded = true;
    c->failed = false;
    return UHNSW_OK;
}

int uhnsw_load_graphs(uhnsw_ctx *c, const uhnsw_index *idx) {
    const auto body = [&] { return load_graphs_body(c, idx); };
    return no_throw("uhnsw_load_graphs", body, [&](const char *w) { if (c) ctx_set_error(c, w); });
}

static int load_graph_files_body(uhnsw_ctx *c, const char *vec_path, const char *g1_path, const char *g2_path,
                                 int32_t storage, int32_t variant) {
    if (!c) return UHNSW_EINVAL;
    IndexFiles f;
    int r = read_index_files(&c->err, vec_path, g1_path, g2_path, storage, variant, &f);
    return r ? r : uhnsw_load_graphs(c, &f.idx);
}

int uhnsw_load_graph_files(uhnsw_ctx *c, const char *vec_path, const char *g1_path, const char *g2_path,
                           int32_t storage, int32_t variant) {
    const auto body = [&] { return load_graph_files_body(c, vec_path, g1_path, g2_path, storage, variant); };
    return no_throw("uhnsw_load_graph_files", body, [&](const char *w) { if (c) ctx_set_error(c, w); });
}

static int check_index_body(const uhnsw_index *idx, char *msg, int32_t msg_len) {
    std::string err;
    return check_result(err, check_index(&err, idx), msg, msg_len);
}

int uhnsw_check_index(const uhnsw_index *idx, char *msg, int32_t msg_len) {
    const auto body = [&] { return check_index_body(idx, msg, msg_len); };
    return no_throw("uhnsw_check_index", body, [&](const char *w) {
        if (msg && msg_len > 0) std::snprintf(msg, (size_t)msg_len, "%s", w);
    });
}

static int check_index_files_body(const char *vec_path, const char *g1_path, const char *g2_path, int32_t storage,
                                  int32_t variant, char *msg, int32_t msg_len) {
    std::string err;
    IndexFiles f;
    int r = read_index_files(&err, vec_path, g1_path, g2_path, storage, variant, &f);
    if (!r) r = check_index(&err, &f.idx);
    return check_result(err, r, msg, msg_len);
}

int uhnsw_check_index_files(const char *vec_path, const char *g1_path, const char *g2_path, int32_t storage,
                            int32_t variant, char *msg, int32_t msg_len) {
    const auto body = [&] {
        return check_index_files_body(vec_path, g1_path, g2_path, storage, variant, msg, msg_len);
    };
    return no_throw("uhnsw_check_index_files", body, [&](const char *w) {
        if (msg && msg_len > 0) std::snprintf(msg, (size_t)msg_len, "%s", w);
    });
}

int uhnsw_get_layout(const uhnsw_ctx *c, int32_t *g, int32_t *v) {
    if (!c || !g || !v) return UHNSW_EINVAL;
    if (!c->loaded) return UHNSW_ESTATE;
    const LayoutInfo li = layout_info(c->layout);
    *g = li.G;
    *v = li.V;
    return UHNSW_OK;
}

int uhnsw_device_info(const uhnsw_ctx *c_, int32_t *num_cus, int32_t *wall_clock_khz) {
    uhnsw_ctx *c = const_cast<uhnsw_ctx *>(c_);
    if (!c || !num_cus || !wall_clock_khz) return UHNSW_EINVAL;
    int rate = 0;
    HIP_OR_FAIL(c, hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, c->device));
    *num_cus = c->num_cus;
    *wall_clock_khz = rate;
    return UHNSW_OK;
}

int uhnsw_last_timing_split(const uhnsw_ctx *c_, float *prepass_ms, float *walk_ms, float *verify_ms) {
    uhnsw_ctx *c = const_cast<uhnsw_ctx *>(c_);
    if (!c || !prepass_ms || !walk_ms || !verify_ms) return UHNSW_EINVAL;
    const auto *S = c->last_set;
    if (!S || !S->timed) return fail(c, UHNSW_ESTATE, "no timed search yet");
    if (!S->split) return fail(c, UHNSW_ESTATE, "the last timed search was a graph replay: no split");
    HIP_OR_FAIL(c, hipEventSynchronize(S->ev[2]));
    HIP_OR_FAIL(c, hipEventElapsedTime(prepass_ms, S->ev[0], S->ev[3]));
    HIP_OR_FAIL(c, hipEventElapsedTime(walk_ms, S->ev[3], S->ev[1]));
    HIP_OR_FAIL(c, hipEventElapsedTime(verify_ms, S->ev[1], S->ev[2]));
    return UHNSW_OK;
}

int uhnsw_last_timing(const uhnsw_ctx *c_, float *walk_ms, float *verify_ms) {
    uhnsw_ctx *c = const_cast<uhnsw_ctx *>(c_);
    if (!c || !walk_ms || !verify_ms) return UHNSW_EINVAL;
    const auto *S = c->last_set;
    if (!S || !S->timed) return fail(c, UHNSW_ESTATE, "no timed search yet");
    HIP_OR_FAIL(c, hipEventSynchronize(S->ev[2]));
    HIP_OR_FAIL(c, hipEventElapsedTime(walk_ms, S->ev[0], S->ev[1]));
    HIP_OR_FAIL(c, hipEventElapsedTime(verify_ms, S->ev[1], S->ev[2]));
    return UHNSW_OK;
}

// (S is the set of the stream the work finally runs on; under capture
// `stream` is the capture stream.)
// Scratch of one search besides the caller's outputs: default stats, the
// two-kernel path's candidate lists, the work counter, the pre-pass arrays.
struct Scratch {
    uhnsw_stats *stats = nullptr;
    int32_t *cand_ids = nullptr, *ncand = nullptr, *counter = nullptr;
    float *cand_keys = nullptr;
    int32_t *o_entry = nullptr, *o_dnb = nullptr, *o_order = nullptr, *o_misc = nullptr;
    float *o_ekey = nullptr, *o_dist = nullptr;
};

// One search enqueued on `stream`. Scratch comes from the stream's set S
// (allocated or grown on demand), or, when `fixed` is given (S is then
// null), is carved from that device region of `fixed_bytes` bytes: no
// allocation, no events, no graph capture.
static int search_on(uhnsw_ctx *c, uhnsw_ctx::StreamSet *S, const float *queries, int64_t nq, const float *p,
                     const int32_t *k, const int32_t *ef, int32_t k_max, int32_t ef_max, const uhnsw_params *prm_in,
                     int32_t k_stride, int64_t *ids, float *dists, uhnsw_stats *stats, int32_t *cand_ids,
                     float *cand_keys, int32_t c_stride, void *stream, void *fixed = nullptr,
                     size_t fixed_bytes = 0) {
    if (c->failed) return fail(c, UHNSW_ESTATE, "context failed earlier: %s", c->err.c_str());
    if (!c->loaded) return fail(c, UHNSW_ESTATE, "no index loaded");
    if (nq < 0 || nq > INT32_MAX) return fail(c, UHNSW_EINVAL, "nq=%lld outside [0, 2^31)", (long long)nq);
    if (nq == 0) return UHNSW_OK;
    if (!queries || !p || !k || !ef || !ids || !dists) return fail(c, UHNSW_EINVAL, "NULL array argument");
    if (k_max < 1 || k_max > UHNSW_KMAX) return fail(c, UHNSW_EINVAL, "k_max=%d outside [1, %d]", k_max, UHNSW_KMAX);
    if (ef_max < k_max || ef_max > UHNSW_EFMAX)
        return fail(c, UHNSW_EINVAL, "ef_max=%d outside [k_max, %d]", ef_max, UHNSW_EFMAX);
    if (k_stride < k_max) return fail(c, UHNSW_EINVAL, "k_stride=%d < k_max=%d", k_stride, k_max);
    if ((cand_ids || cand_keys) && (!cand_ids || !cand_keys || c_stride < ef_max))
        return fail(c, UHNSW_EINVAL, "candidate output needs both arrays and c_stride >= ef_max");
    uhnsw_params prm;
    if (prm_in)
        prm = *prm_in;
    else
        uhnsw_default_params(&prm);
    int r = check_params(c, prm);
    if (r) return r;
    Plan pl;
    if ((r = make_plan(c, k_max, ef_max, prm, &pl))) return r;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_OR_FAIL(c, hipSetDevice(c->device));

    SearchArgs a{};
    a.walk_base = c->storage == UHNSW_STORE_F32 ? c->f32_base.p : c->walk_base.p;
    a.f32_base = c->f32_base.as<float>();
    a.pitch = c->pitch;
    a.n = (int32_t)c->n;
    a.d = c->d;
    a.storage = c->storage;
    for (int i = 0; i < 2; ++i) {
        a.g[i].adj0 = c->g[i].adj0.as<int32_t>();
        a.g[i].up_off = c->g[i].up_off.as<int32_t>();
        a.g[i].up_adj = c->g[i].up_adj.as<int32_t>();
        a.g[i].entry = c->g[i].entry;
        a.g[i].max_level = c->g[i].max_level;
        a.g[i].M = c->g[i].M;
        a.g[i].M0 = c->g[i].M0;
    }
    a.queries = queries;
    a.p = p;
    a.k = k;
    a.ef = ef;
    a.nq = nq;
    a.k_max = k_max;
    a.ef_max = ef_max;
    // Sec. 3.1's 1.4, Sec. 4.5's 0.6 for the extended pair; the per-p graph
    // takes every query
    a.cutoff = prm.cutoff > 0.0f ? prm.cutoff
               : c->variant == UHNSW_VARIANT_EXT ? 0.6f
               : c->variant == UHNSW_VARIANT_PGRAPH ? INFINITY
                                                     : 1.4f;
    a.ext = c->variant != UHNSW_VARIANT_STD;
    a.walk_p = c->graph_p;
    p_range(c->variant, &a.p_lo, &a.p_hi);
    a.l05_fast = c->l05_fast;
    a.l05_table = c->l05_table;
    a.t_param = prm.t;
    a.kappa_param = prm.kappa;
    a.beam = prm.beam_width;
    a.early_abort = prm.early_abort;
    fill_mtab(prm.tau, a.mtab);
    a.ef_cap = pl.ef_cap;
    a.vis_bits = pl.vis_bits;
    a.vis_kbits = pl.vis_kbits;
    a.kv_cap = pl.kv_cap;
    a.waves_per_block = pl.wpb;
    a.ids = ids;
    a.dists = dists;
    a.k_stride = k_stride;
    a.counter = nullptr;
    a.order = nullptr;
    const bool ordered = prm.persistent >= 2;
    const bool counted = prm.persistent == 1 || prm.persistent == 2;  // 3: ordered static grid
    const int32_t cs = prm.fused ? (cand_ids ? c_stride : 0) : (cand_ids ? c_stride : ef_max);
    const bool own_cand = !prm.fused && !cand_ids;
    Scratch sc;
    if (fixed) {
        if (prm.graph || prm.timing)
            return fail(c, UHNSW_EINVAL, "graph capture and timing need allocations: not in this entry point");
        // carve the region in 256-byte aligned pieces, in a fixed order
        size_t off = 0;
        auto take = [&](size_t bytes) -> void * {
            off = (off + 255) & ~(size_t)255;
            void *q = static_cast<char *>(fixed) + off;
            off += bytes;
            return q;
        };
        const size_t q4 = (size_t)nq * 4;
        if (!stats) sc.stats = static_cast<uhnsw_stats *>(take((size_t)nq * sizeof(uhnsw_stats)));
        if (own_cand) {
            sc.cand_ids = static_cast<int32_t *>(take((size_t)nq * cs * 4));
            sc.cand_keys = static_cast<float *>(take((size_t)nq * cs * 4));
        }
        if (!prm.fused) sc.ncand = static_cast<int32_t *>(take(q4));
        if (counted) sc.counter = static_cast<int32_t *>(take(4));
        if (ordered) {
            sc.o_entry = static_cast<int32_t *>(take(q4));
            sc.o_ekey = static_cast<float *>(take(q4));
            sc.o_dnb = static_cast<int32_t *>(take(q4));
            sc.o_dist = static_cast<float *>(take(q4));
            sc.o_order = static_cast<int32_t *>(take(q4));
            sc.o_misc = static_cast<int32_t *>(take((6 + 2 * kOrderBuckets) * 4));
        }
        if (off > fixed_bytes)
            return fail(c, UHNSW_EINVAL,
                        "this search needs %zu bytes of scratch, above the fixed region's %zu (fewer queries, a "
                        "smaller ef_max, the fused kernel or caller-held stats need less)",
                        off, fixed_bytes);
    } else {
        const size_t q4 = (size_t)nq * 4;
        if (!stats) {
            HIP_OR_FAIL(c, ensure_scratch(c, S->stats, (size_t)nq * sizeof(uhnsw_stats)));
            sc.stats = S->stats.as<uhnsw_stats>();
        }
        if (own_cand) {
            HIP_OR_FAIL(c, ensure_scratch(c, S->cand_ids, (size_t)nq * cs * 4));
            HIP_OR_FAIL(c, ensure_scratch(c, S->cand_keys, (size_t)nq * cs * 4));
            sc.cand_ids = S->cand_ids.as<int32_t>();
            sc.cand_keys = S->cand_keys.as<float>();
        }
        if (!prm.fused) {
            HIP_OR_FAIL(c, ensure_scratch(c, S->ncand, q4));
            sc.ncand = S->ncand.as<int32_t>();
        }
        if (counted) {
            HIP_OR_FAIL(c, ensure_scratch(c, S->counter, 4));
            sc.counter = S->counter.as<int32_t>();
        }
        if (ordered) {
            HIP_OR_FAIL(c, ensure_scratch(c, S->o_entry, q4));
            HIP_OR_FAIL(c, ensure_scratch(c, S->o_ekey, q4));
            HIP_OR_FAIL(c, ensure_scratch(c, S->o_dnb, q4));
            HIP_OR_FAIL(c, ensure_scratch(c, S->o_dist, q4));
            HIP_OR_FAIL(c, ensure_scratch(c, S->o_order, q4));
            HIP_OR_FAIL(c, ensure_scratch(c, S->o_misc, (6 + 2 * kOrderBuckets) * 4));
            sc.o_entry = S->o_entry.as<int32_t>();
            sc.o_ekey = S->o_ekey.as<float>();
            sc.o_dnb = S->o_dnb.as<int32_t>();
            sc.o_dist = S->o_dist.as<float>();
            sc.o_order = S->o_order.as<int32_t>();
            sc.o_misc = S->o_misc.as<int32_t>();
        }
    }
    a.stats = stats ? stats : sc.stats;
    a.cand_ids = cand_ids ? cand_ids : sc.cand_ids;  // fused: C stays in LDS unless the caller asks for it
    a.cand_keys = cand_ids ? cand_keys : sc.cand_keys;
    a.c_stride = cs;
    a.ncand = sc.ncand;
    OrderArgs oa{};
    if (ordered) {
        oa.entry = sc.o_entry;
        oa.ekey = sc.o_ekey;
        oa.dnb = sc.o_dnb;
        oa.dist = sc.o_dist;
        oa.gsum = reinterpret_cast<float *>(sc.o_misc);
        oa.bcnt = sc.o_misc + 6;
        oa.order = sc.o_order;
    }

    // the kernels of one search, in stream order
    const int grid_all = (int)((nq + pl.wpb - 1) / pl.wpb);
    int pgrid = grid_all;
    if (counted) {
        int per_cu = 0;
        const void *kp =
            prm.fused ? search_kernel_ptr(c->layout, c->storage, prm.beam_width, a.ext != 0)
                      : walk_kernel_ptr(c->layout, c->storage, a.ext != 0);
        const size_t lds_block = (size_t)(prm.fused ? pl.search_bytes : pl.walk_bytes) * pl.wpb;
        bool found = false;
        for (auto &o : c->occ)
            if (o.kernel == kp && o.block == pl.wpb * kWave && o.lds == lds_block) {
                per_cu = o.per_cu;
                found = true;
            }
        if (!found) {
            HIP_OR_FAIL(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kp, pl.wpb * kWave, lds_block));
            if (!fixed) c->occ.push_back({kp, pl.wpb * kWave, lds_block, per_cu});
        }
        per_cu = std::max(per_cu, 1);
        if (prm.waves_per_cu > 0) per_cu = std::min(per_cu, std::max(1, prm.waves_per_cu / pl.wpb));
        pgrid = std::max(1, std::min(grid_all, per_cu * c->num_cus));
    }
    auto enqueue = [&](hipStream_t st, bool timed) -> hipError_t {
        hipError_t e = hipSuccess;
        SearchArgs b = a;
        if (counted) {
            b.counter = sc.counter;
            if ((e = launch_fill_i32(b.counter, 0, 1, st)) != hipSuccess) return e;
        }
        if (timed && (e = hipEventRecord(S->ev[0], st)) != hipSuccess) return e;
        if (ordered) {  // descent pre-pass, then the likely-long queries first
            if ((e = launch_fill_i32(sc.o_misc, 0, 6 + 2 * kOrderBuckets, st)) != hipSuccess) return e;
            if ((e = launch_order(b, oa, c->layout, st)) != hipSuccess) return e;
            b.order = oa.order;
            b.entry = oa.entry;
            b.ekey = oa.ekey;
            b.dnb = oa.dnb;
        }
        if (timed && (e = hipEventRecord(S->ev[3], st)) != hipSuccess) return e;
        if (prm.fused) {
            b.lds_wave_bytes = pl.search_bytes;
            if ((e = launch_search(b, c->layout, counted ? pgrid : grid_all, st)) != hipSuccess) return e;
            if (timed && (e = hipEventRecord(S->ev[1], st)) != hipSuccess) return e;
        } else {
            b.lds_wave_bytes = pl.walk_bytes;
            if ((e = launch_walk(b, c->layout, counted ? pgrid : grid_all, st)) != hipSuccess) return e;
            if (timed && (e = hipEventRecord(S->ev[1], st)) != hipSuccess) return e;
            b.lds_wave_bytes = pl.verify_bytes;
            b.counter = nullptr;
            if ((e = launch_verify(b, c->layout, grid_all, st)) != hipSuccess) return e;
        }
        if (timed && (e = hipEventRecord(S->ev[2], st)) != hipSuccess) return e;
        return hipSuccess;
    };

    if (fixed) {
        HIP_OR_FAIL(c, enqueue(s, false));
        return UHNSW_OK;
    }
    S->timed = prm.timing != 0;
    S->split = S->timed && !prm.graph;
    c->last_set = S;
    if (!prm.graph) {
        HIP_OR_FAIL(c, enqueue(s, S->timed));
        return UHNSW_OK;
    }
    // hipGraph: capture the launch sequence once per distinct argument set,
    // replay it afterwards (kernel arguments are baked into the graph)
    GraphKey key{};
    key.ptrs[0] = queries;
    key.ptrs[1] = p;
    key.ptrs[2] = k;
    key.ptrs[3] = ef;
    key.ptrs[4] = ids;
    key.ptrs[5] = dists;
    key.ptrs[6] = stats;
    key.ptrs[7] = cand_ids;
    key.ptrs[8] = cand_keys;
    key.nq = nq;
    key.ints[0] = k_max;
    key.ints[1] = ef_max;
    key.ints[2] = k_stride;
    key.ints[3] = c_stride;
    key.prm = prm;
    key.prm.timing = 0;
    key.prm.graph = 0;
    key.gen = c->scratch_gen;
    if (!S->gexec || std::memcmp(&key, &S->gkey, sizeof key) != 0) {
        if (S->gexec) {
            (void)hipGraphExecDestroy(S->gexec);
            S->gexec = nullptr;
        }
        if (!c->cap_stream) HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        HIP_OR_FAIL(c, hipStreamSynchronize(s));
        HIP_OR_FAIL(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue(c->cap_stream, false);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
        if (e != hipSuccess) return dev_fail(c, e, "enqueue under capture");
        if (e2 != hipSuccess) return dev_fail(c, e2, "hipStreamEndCapture");
        e = hipGraphInstantiate(&S->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return dev_fail(c, e, "hipGraphInstantiate");
        S->gkey = key;
        ++c->graph_captures;
    }
    if (S->timed) HIP_OR_FAIL(c, hipEventRecord(S->ev[0], s));
    HIP_OR_FAIL(c, hipGraphLaunch(S->gexec, s));
    if (S->timed) {
        HIP_OR_FAIL(c, hipEventRecord(S->ev[1], s));
        HIP_OR_FAIL(c, hipEventRecord(S->ev[2], s));
    }
    return UHNSW_OK;
}

// The scratch set of a launch stream, created on first use.
static int stream_set(uhnsw_ctx *c, hipStream_t st, uhnsw_ctx::StreamSet **out) {
    for (auto &S : c->sets)
        if (S->stream == st) {
            *out = S.get();
            return UHNSW_OK;
        }
    if (c->sets.size() >= (size_t)kMaxStreams)
        return fail(c, UHNSW_EUNSUPPORTED, "searches on more than %d streams per context", kMaxStreams);
    auto S = std::make_unique<uhnsw_ctx::StreamSet>();
    S->stream = st;
    for (auto &ev : S->ev) HIP_OR_FAIL(c, hipEventCreate(&ev));
    *out = S.get();
    c->sets.push_back(std::move(S));
    return UHNSW_OK;
}

static int search_device_body(uhnsw_ctx *c, const float *queries, int64_t nq, const float *p, const int32_t *k,
                              const int32_t *ef, int32_t k_max, int32_t ef_max, const uhnsw_params *prm_in,
                              int32_t k_stride, int64_t *ids, float *dists, uhnsw_stats *stats, int32_t *cand_ids,
                              float *cand_keys, int32_t c_stride, void *stream) {
    if (!c) return UHNSW_EINVAL;
    if (c->failed) return fail(c, UHNSW_ESTATE, "context failed earlier: %s", c->err.c_str());
    uhnsw_ctx::StreamSet *S = nullptr;
    HIP_OR_FAIL(c, hipSetDevice(c->device));
    if (int r = stream_set(c, reinterpret_cast<hipStream_t>(stream), &S)) return r;
    return search_on(c, S, queries, nq, p, k, ef, k_max, ef_max, prm_in, k_stride, ids, dists, stats, cand_ids,
                     cand_keys, c_stride, stream);
}

int uhnsw_search_device(uhnsw_ctx *c, const float *queries, int64_t nq, const float *p, const int32_t *k,
                        const int32_t *ef, int32_t k_max, int32_t ef_max, const uhnsw_params *prm_in,
                        int32_t k_stride, int64_t *ids, float *dists, uhnsw_stats *stats, int32_t *cand_ids,
                        float *cand_keys, int32_t c_stride, void *stream) {
    const auto body = [&] {
        return search_device_body(c, queries, nq, p, k, ef, k_max, ef_max, prm_in, k_stride, ids, dists, stats,
                                  cand_ids, cand_keys, c_stride, stream);
    };
    return no_throw("uhnsw_search_device", body, [&](const char *w) { if (c) ctx_set_error(c, w); });
}

static int search_device_noalloc_body(uhnsw_ctx *c, const float *queries, int64_t nq, const float *p, const int32_t *k,
                                      const int32_t *ef, int32_t k_max, int32_t ef_max, const uhnsw_params *prm_in,
                                      int32_t k_stride, int64_t *ids, float *dists, uhnsw_stats *stats,
                                      int32_t *cand_ids, float *cand_keys, int32_t c_stride, void *stream) {
    if (!c) return UHNSW_EINVAL;
    if (!c->noalloc) return fail(c, UHNSW_ESTATE, "no fixed scratch region on device %d", c->device);
    return search_on(c, nullptr, queries, nq, p, k, ef, k_max, ef_max, prm_in, k_stride, ids, dists, stats,
                     cand_ids, cand_keys, c_stride, stream, c->noalloc, kNoAllocScratchBytes);
}

int uhnsw_search_device_noalloc(uhnsw_ctx *c, const float *queries, int64_t nq, const float *p, const int32_t *k,
                                const int32_t *ef, int32_t k_max, int32_t ef_max, const uhnsw_params *prm_in,
                                int32_t k_stride, int64_t *ids, float *dists, uhnsw_stats *stats,
                                int32_t *cand_ids, float *cand_keys, int32_t c_stride, void *stream) {
    const auto body = [&] {
        return search_device_noalloc_body(c, queries, nq, p, k, ef, k_max, ef_max, prm_in, k_stride, ids, dists,
                                          stats, cand_ids, cand_keys, c_stride, stream);
    };
    return no_throw("uhnsw_search_device_noalloc", body, [&](const char *w) { if (c) ctx_set_error(c, w); });
}

static int probe_gather_body(uhnsw_ctx *c, int32_t row_bytes, double *gbs) {
    if (!c || !gbs) return UHNSW_EINVAL;
    if (!c->loaded) return fail(c, UHNSW_ESTATE, "no index loaded");
    if (row_bytes != 128 && row_bytes != 256 && row_bytes != 512)
        return fail(c, UHNSW_EINVAL, "row_bytes=%d not 128, 256 or 512", row_bytes);
    if ((int64_t)row_bytes > c->pitch * 4)
        return fail(c, UHNSW_EINVAL, "row_bytes=%d above the row pitch (%lld B)", row_bytes,
                    (long long)(c->pitch * 4));
    HIP_OR_FAIL(c, hipSetDevice(c->device));
    DevBuf sink;
    HIP_OR_FAIL(c, sink.ensure(4));
    const int blocks = c->num_cus * 8;  // 32 waves per CU requested, the hardware keeps what fits
    const int iters = 256;
    hipEvent_t e0, e1;
    HIP_OR_FAIL(c, hipEventCreate(&e0));
    HIP_OR_FAIL(c, hipEventCreate(&e1));
    hipError_t e = launch_gather_probe(c->f32_base.as<float>(), c->n, c->pitch, row_bytes, blocks, iters, 1u,
                                       sink.as<float>(), c->stream);  // warm-up
    float best = 1e30f;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
        float ms = 0;
        if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) break;
        if ((e = launch_gather_probe(c->f32_base.as<float>(), c->n, c->pitch, row_bytes, blocks, iters,
                                     2u + (uint32_t)rep, sink.as<float>(), c->stream)) != hipSuccess)
            break;
        if ((e = hipEventRecord(e1, c->stream)) != hipSuccess) break;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return dev_fail(c, e, "gather probe");
    const double bytes = (double)blocks * 4 * iters * 32 * row_bytes;
    *gbs = bytes / (best * 1e-3) / 1e9;
    return UHNSW_OK;
}

int uhnsw_probe_gather(uhnsw_ctx *c, int32_t row_bytes, double *gbs) {
    const auto body = [&] { return probe_gather_body(c, row_bytes, gbs); };
    return no_throw("uhnsw_probe_gather", body, [&](const char *w) { if (c) ctx_set_error(c, w); });
}

static int probe_transcendental_body(uhnsw_ctx *c, double *ops_per_s) {
    if (!c || !ops_per_s) return UHNSW_EINVAL;
    HIP_OR_FAIL(c, hipSetDevice(c->device));
    DevBuf sink;
    HIP_OR_FAIL(c, sink.ensure(4));
    const int blocks = c->num_cus * 8;
    const int iters = 256;
    hipEvent_t e0, e1;
    HIP_OR_FAIL(c, hipEventCreate(&e0));
    HIP_OR_FAIL(c, hipEventCreate(&e1));
    hipError_t e = launch_trans_probe(blocks, iters, sink.as<float>(), c->stream);
    float best = 1e30f;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
        float ms = 0;
        if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) break;
        if ((e = launch_trans_probe(blocks, iters, sink.as<float>(), c->stream)) != hipSuccess) break;
        if ((e = hipEventRecord(e1, c->stream)) != hipSuccess) break;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return dev_fail(c, e, "transcendental probe");
    const double ops = (double)blocks * 256 * iters * 8 * 2;  // one v_log and one v_exp per chain step
    *ops_per_s = ops / (best * 1e-3);
    return UHNSW_OK;
}

int uhnsw_probe_transcendental(uhnsw_ctx *c, double *ops_per_s) {
    const auto body = [&] { return probe_transcendental_body(c, ops_per_s); };
    return no_throw("uhnsw_probe_transcendental", body, [&](const char *w) { if (c) ctx_set_error(c, w); });
}

int uhnsw_graph_captures(const uhnsw_ctx *c, int64_t *count) {
    if (!c || !count) return UHNSW_EINVAL;
    *count = c->graph_captures;
    return UHNSW_OK;
}

static int autotune_body(uhnsw_ctx *c, const float *queries, int64_t nq, const float *p, const int32_t *k,
                         const int32_t *ef, int32_t k_max, int32_t ef_max, int32_t flags, uhnsw_params *prm,
                         void *stream) {
    if (!c || !prm) return UHNSW_EINVAL;
    if (!c->loaded) return fail(c, UHNSW_ESTATE, "no index loaded");
    if (nq < 1) return fail(c, UHNSW_EINVAL, "autotune needs queries");
    const uint64_t key = ((uint64_t)c->n << 20) ^ ((uint64_t)c->d << 8) ^ ((uint64_t)c->storage << 4) ^
                         ((uint64_t)(ef_max <= 64 ? 0 : ef_max <= 128 ? 1 : ef_max <= 256 ? 2 : 3) << 40) ^
                         ((uint64_t)k_max << 44) ^ ((uint64_t)(flags & 3) << 58) ^
                         ((uint64_t)(prm->fused != 0) << 61) ^ ((uint64_t)c->variant << 62);
    const bool allow_beam = (flags & UHNSW_TUNE_BEAM) != 0;
    const bool pipelined = (flags & UHNSW_TUNE_PIPELINED) != 0;
    for (auto &e : c->tuned)
        if (e.first == key) {
            uhnsw_params t = e.second;
            t.tau = prm->tau;
            t.cutoff = prm->cutoff;
            t.t = prm->t;
            t.kappa = prm->kappa;
            t.early_abort = prm->early_abort;
            t.timing = prm->timing;
            t.graph = prm->graph;
            *prm = t;
            return UHNSW_OK;
        }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    DevBuf oid[2], od[2], os[2];
    for (int j = 0; j < (pipelined ? 2 : 1); ++j) {
        HIP_OR_FAIL(c, oid[j].ensure((size_t)nq * k_max * 8));
        HIP_OR_FAIL(c, od[j].ensure((size_t)nq * k_max * 4));
        HIP_OR_FAIL(c, os[j].ensure((size_t)nq * sizeof(uhnsw_stats)));
    }
    // the second stream of the pipelined timing: the context's own stream
    // unless the caller's is that one
    if (pipelined && s == c->stream && !c->tune_stream)
        HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->tune_stream, hipStreamNonBlocking));
    hipStream_t st2[2] = {s, s == c->stream ? c->tune_stream : c->stream};
    uhnsw_params best = *prm;
    float best_ms = 1e30f;
    // median of three timed runs (after one untimed) of the knobs in t;
    // returns 1 when the shape does not fit (skipped), 0 or an error code
    auto measure = [&](uhnsw_params t, float *median_ms) -> int {
        t.graph = 0;
        t.timing = 1;
        float ms[3];
        for (int rep = -1; rep < 3; ++rep) {
            if (pipelined) {  // 6 launches, two in flight: wall time per launch
                t.timing = 0;
                if (rep >= 0) HIP_OR_FAIL(c, hipStreamSynchronize(s));
                const auto t0 = std::chrono::steady_clock::now();
                for (int l = 0; l < 6; ++l) {
                    const int j = l & 1;
                    int rc = uhnsw_search_device(c, queries, nq, p, k, ef, k_max, ef_max, &t, k_max,
                                                 oid[j].as<int64_t>(), od[j].as<float>(), os[j].as<uhnsw_stats>(),
                                                 nullptr, nullptr, 0, st2[j]);
                    if (rc == UHNSW_EUNSUPPORTED || rc == UHNSW_EINVAL) {
                        c->err.clear();
                        HIP_OR_FAIL(c, hipStreamSynchronize(st2[0]));
                        HIP_OR_FAIL(c, hipStreamSynchronize(st2[1]));
                        return 1;
                    }
                    if (rc) return rc;
                }
                HIP_OR_FAIL(c, hipStreamSynchronize(st2[0]));
                HIP_OR_FAIL(c, hipStreamSynchronize(st2[1]));
                const double dt =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                if (rep >= 0) ms[rep] = (float)(dt / 6);
                continue;
            }
            int rc = uhnsw_search_device(c, queries, nq, p, k, ef, k_max, ef_max, &t, k_max, oid[0].as<int64_t>(),
                                         od[0].as<float>(), os[0].as<uhnsw_stats>(), nullptr, nullptr, 0, s);
            if (rc == UHNSW_EUNSUPPORTED || rc == UHNSW_EINVAL) {
                c->err.clear();  // this shape does not fit: skip it
                return 1;
            }
            if (rc) return rc;
            float w = 0, v = 0;
            if ((rc = uhnsw_last_timing(c, &w, &v))) return rc;
            if (rep >= 0) ms[rep] = w + v;
        }
        std::sort(ms, ms + 3);
        *median_ms = ms[1];
        return 0;
    };
    const int slots_c[] = {1024, 2048, 4096};
    const int wpb_c[] = {1, 2, 4};
    for (int beam = 1; beam <= (allow_beam ? 2 : 1); ++beam)
        for (int sl : slots_c)
            for (int wpb : wpb_c)
                for (int pers = 0; pers <= 3; ++pers) {
                    uhnsw_params t = *prm;
                    t.beam_width = beam;
                    t.visited_slots = sl;
                    t.waves_per_block = wpb;
                    t.persistent = pers;
                    t.waves_per_cu = 0;
                    float ms = 0.0f;
                    const int r = measure(t, &ms);
                    if (r < 0) return r;
                    if (r == 0 && ms < best_ms) {
                        best_ms = ms;
                        best = t;
                    }
                }
    // queries per CU: a persistent launch may do better with fewer resident
    // waves than fit (less contention for the caches and HBM queues)
    if (best.persistent == 1 || best.persistent == 2) {
        const uhnsw_params base = best;
        for (int wcu : {8, 12}) {
            uhnsw_params t = base;
            t.waves_per_cu = wcu;
            float ms = 0.0f;
            const int r = measure(t, &ms);
            if (r < 0) return r;
            if (r == 0 && ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    }
    best.timing = prm->timing;
    best.graph = prm->graph;
    c->tuned.emplace_back(key, best);
    *prm = best;
    return UHNSW_OK;
}

int uhnsw_autotune(uhnsw_ctx *c, const float *queries, int64_t nq, const float *p, const int32_t *k,
                   const int32_t *ef, int32_t k_max, int32_t ef_max, int32_t flags, uhnsw_params *prm,
                   void *stream) {
    const auto body = [&] { return autotune_body(c, queries, nq, p, k, ef, k_max, ef_max, flags, prm, stream); };
    return no_throw("uhnsw_autotune", body, [&](const char *w) { if (c) ctx_set_error(c, w); });
}

static int search_body(uhnsw_ctx *c, const float *queries, int64_t nq, const float *p, const int32_t *k,
                       const int32_t *ef, const uhnsw_params *prm_in, int32_t k_stride, int64_t *ids, float *dists,
                       uhnsw_stats *stats) {
    if (!c) return UHNSW_EINVAL;
    if (c->failed) return fail(c, UHNSW_ESTATE, "context failed earlier: %s", c->err.c_str());
    if (!c->loaded) return fail(c, UHNSW_ESTATE, "no index loaded");
    if (nq < 0 || nq > INT32_MAX) return fail(c, UHNSW_EINVAL, "nq=%lld outside [0, 2^31)", (long long)nq);
    if (nq == 0) return UHNSW_OK;
    if (!queries || !p || !k || !ef || !ids || !dists) return fail(c, UHNSW_EINVAL, "NULL array argument");
    int k_max = 0, ef_max = 0;
    for (int64_t i = 0; i < nq; ++i) {
        if (!std::isfinite(p[i]) || !p_in_range(c->variant, p[i]))
            return fail(c, UHNSW_EINVAL, "p[%lld]=%g outside %s", (long long)i, (double)p[i],
                        c->variant == UHNSW_VARIANT_EXT ? "[0.2, 1]"
                        : c->variant == UHNSW_VARIANT_PGRAPH ? "[0.2, 2]" : "[0.5, 2]");
        if (k[i] < 1 || k[i] > UHNSW_KMAX)
            return fail(c, UHNSW_EINVAL, "k[%lld]=%d outside [1, %d]", (long long)i, k[i], UHNSW_KMAX);
        if (ef[i] < k[i] || ef[i] > UHNSW_EFMAX)
            return fail(c, UHNSW_EINVAL, "ef[%lld]=%d outside [k, %d]", (long long)i, ef[i], UHNSW_EFMAX);
        k_max = std::max(k_max, k[i]);
        ef_max = std::max(ef_max, ef[i]);
    }
    for (int64_t i = 0; i < nq * c->d; ++i)
        if (!std::isfinite(queries[i]))
            return fail(c, UHNSW_EINVAL, "query value %lld is not finite", (long long)i);
    if (k_stride < k_max) return fail(c, UHNSW_EINVAL, "k_stride=%d < max k=%d", k_stride, k_max);
    HIP_OR_FAIL(c, hipSetDevice(c->device));
    const size_t nqs = (size_t)nq;
    HIP_OR_FAIL(c, ensure_scratch(c, c->s_q, nqs * c->d * 4));
    HIP_OR_FAIL(c, ensure_scratch(c, c->s_p, nqs * 4));
    HIP_OR_FAIL(c, ensure_scratch(c, c->s_k, nqs * 4));
    HIP_OR_FAIL(c, ensure_scratch(c, c->s_ef, nqs * 4));
    HIP_OR_FAIL(c, ensure_scratch(c, c->s_ids, nqs * k_stride * 8));
    HIP_OR_FAIL(c, ensure_scratch(c, c->s_dists, nqs * k_stride * 4));
    HIP_OR_FAIL(c, ensure_scratch(c, c->s_stats, nqs * sizeof(uhnsw_stats)));
    hipStream_t s = c->stream;
    uhnsw_ctx::StreamSet *S = nullptr;
    if (int r = stream_set(c, s, &S)) return r;
    uhnsw_params prm;
    if (prm_in)
        prm = *prm_in;
    else
        uhnsw_default_params(&prm);
    const size_t bytes[7] = {nqs * c->d * 4, nqs * 4, nqs * 4, nqs * 4, nqs * k_stride * 8, nqs * k_stride * 4,
                             nqs * sizeof(uhnsw_stats)};
    void *dev[7] = {c->s_q.p, c->s_p.p, c->s_k.p, c->s_ef.p, c->s_ids.p, c->s_dists.p, c->s_stats.p};
    // the search through one set of host buffers: 4 copies in, kernels, 3 out
    auto enqueue = [&](hipStream_t st, void *const *host, const uhnsw_params &pr) -> int {
        for (int i = 0; i < 4; ++i) HIP_OR_FAIL(c, hipMemcpyAsync(dev[i], host[i], bytes[i], hipMemcpyHostToDevice, st));
        // the scratch of c->stream, also while capturing: the graph runs there
        int r = search_on(c, S, c->s_q.as<float>(), nq, c->s_p.as<float>(), c->s_k.as<int32_t>(),
                          c->s_ef.as<int32_t>(), k_max, ef_max, &pr, k_stride, c->s_ids.as<int64_t>(),
                          c->s_dists.as<float>(), c->s_stats.as<uhnsw_stats>(), nullptr, nullptr, 0, st);
        if (r) return r;
        for (int i = 4; i < 7; ++i) {
            if (i == 6 && !stats) break;
            HIP_OR_FAIL(c, hipMemcpyAsync(host[i], dev[i], bytes[i], hipMemcpyDeviceToHost, st));
        }
        return UHNSW_OK;
    };
    if (!prm.graph) {
        const void *user_in[4] = {queries, p, k, ef};
        void *host[7] = {const_cast<void *>(user_in[0]), const_cast<void *>(user_in[1]),
                         const_cast<void *>(user_in[2]), const_cast<void *>(user_in[3]), ids, dists, stats};
        int r = enqueue(s, host, prm);
        if (r) return r;
        HIP_OR_FAIL(c, hipStreamSynchronize(s));
        return UHNSW_OK;
    }
    // hipGraph: stage through pinned buffers so the captured copies stay valid
    bool grown = false;
    for (int i = 0; i < 7; ++i) {
        if (c->hp[i].bytes >= bytes[i] && c->hp[i].p) continue;
        if (c->hp[i].p) (void)hipHostFree(c->hp[i].p);
        c->hp[i].p = nullptr;
        c->hp[i].bytes = 0;
        HIP_OR_FAIL(c, hipHostMalloc(&c->hp[i].p, bytes[i] ? bytes[i] : 1, hipHostMallocDefault));
        c->hp[i].bytes = bytes[i];
        grown = true;
    }
    void *host[7];
    for (int i = 0; i < 7; ++i) host[i] = c->hp[i].p;
    std::memcpy(host[0], queries, bytes[0]);
    std::memcpy(host[1], p, bytes[1]);
    std::memcpy(host[2], k, bytes[2]);
    std::memcpy(host[3], ef, bytes[3]);
    uhnsw_params pr = prm;
    pr.graph = 0;
    pr.timing = 0;
    GraphKey key{};
    for (int i = 0; i < 7; ++i) key.ptrs[i] = host[i];
    for (int i = 0; i < 7; ++i) key.ptrs[7 + i] = dev[i];
    key.ptrs[14] = reinterpret_cast<const void *>(stats ? 1 : 0);  // whether stats are copied out
    key.nq = nq;
    key.ints[0] = k_max;
    key.ints[1] = ef_max;
    key.ints[2] = k_stride;
    key.prm = pr;
    key.gen = c->scratch_gen;
    if (c->hgexec && !grown && std::memcmp(&key, &c->hgkey, sizeof key) == 0) {
        HIP_OR_FAIL(c, hipGraphLaunch(c->hgexec, s));
        HIP_OR_FAIL(c, hipStreamSynchronize(s));
    } else {
        // first call with this shape: run it, then capture the same sequence
        int r = enqueue(s, host, pr);
        if (r) return r;
        HIP_OR_FAIL(c, hipStreamSynchronize(s));
        if (c->hgexec) {
            (void)hipGraphExecDestroy(c->hgexec);
            c->hgexec = nullptr;
        }
        if (!c->cap_stream) HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        HIP_OR_FAIL(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        r = enqueue(c->cap_stream, host, pr);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
        if (r) return r;
        if (e2 != hipSuccess) return dev_fail(c, e2, "hipStreamEndCapture (host path)");
        hipError_t e = hipGraphInstantiate(&c->hgexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return dev_fail(c, e, "hipGraphInstantiate (host path)");
        key.gen = c->scratch_gen;  // the scratch the captured kernels address
        c->hgkey = key;
        ++c->graph_captures;
    }
    std::memcpy(ids, host[4], bytes[4]);
    std::memcpy(dists, host[5], bytes[5]);
    if (stats) std::memcpy(stats, host[6], bytes[6]);
    return UHNSW_OK;
}

int uhnsw_search(uhnsw_ctx *c, const float *queries, int64_t nq, const float *p, const int32_t *k,
                 const int32_t *ef, const uhnsw_params *prm_in, int32_t k_stride, int64_t *ids, float *dists,
                 uhnsw_stats *stats) {
    const auto body = [&] { return search_body(c, queries, nq, p, k, ef, prm_in, k_stride, ids, dists, stats); };
    return no_throw("uhnsw_search", body, [&](const char *w) { if (c) ctx_set_error(c, w); });
}

}  // extern "C"
