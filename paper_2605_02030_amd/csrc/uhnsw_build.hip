// GPU construction of the HNSW base graphs G1, G2 (and G_0.5, G_p). Building the
// graphs is U-HNSW's up-front cost (Sec. 4.4.3, Table 3); the graph itself is
// HNSW's layered proximity graph (Sec. 2.2). This builds the same graph as
// the deterministic CPU input builder (synth/hnsw_build.c), edge for edge:
//
//   levels   floor(-ln(U_v) / ln M), U_v in (0, 1] from a counter-based
//            draw (splitmix64 of seed ^ v * golden), capped at 30 (host);
//   batches  nodes are inserted in id order, in batches of
//            clamp(nodes_in_graph / 64, 1, batch_max); a batch first plans
//            every member against the graph frozen at the batch start (one
//            wave per member: greedy descent above its level, an
//            efConstruction best-first search on each of its layers, M
//            neighbours per layer by the diversity heuristic, written as
//            its own lists), then applies the reverse links grouped by
//            (layer, target), each target's requests in ascending source id
//            (one wave per target: append, or when the list is full re-select
//            it with the same heuristic);
//   distance FP32 in one fixed order: element j summed by lane (j / 4) mod 16
//            of 16 lanes in ascending j (L2 by fused multiply-add), the lanes
//            combined pairwise (metric 4, sum |x - q|^p for the per-p
//            baseline, takes each term on v_log / v_exp and has no CPU twin).
//
// The layer search is the walk's sorted list with a bounded LDS visited
// cache, which returns the same list as an exact visited set (a forgotten
// node is in the list already or worse than its full worst entry).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "uhnsw_device.h"
#include "uhnsw_guard.h"

namespace uhnsw {
namespace {

constexpr int kBG = 16;            // lanes per row in the build's distance order
constexpr int kBuildLayers = 32;   // levels are capped at 30
constexpr int kLevelCap = 30;

struct BuildArgs {
    const float *base;   // rows of `pitch` floats, zero padded
    int64_t pitch, n;
    int32_t d;
    int32_t *adj0;       // [n * M0], -1 padded
    int32_t *uadj;       // [rows * M], -1 padded
    const int32_t *upo;  // [n] row of layer 1 in uadj, -1 on level-0 nodes
    const int8_t *level; // [n]
    int32_t M, M0, efc;
    int32_t ef_cap, vis_bits, vis_kbits, lds_wave_bytes;
    float metric_p;      // metric 4: the p of sum |x - q|^p
    // plan step
    int64_t done;
    int32_t b, lmax, ep;
    int32_t *plan_ids;   // [b * kBuildLayers * M]
    int32_t *plan_cnt;   // [b * kBuildLayers]
    // link step
    const int32_t *g_l, *g_u, *g_start, *req_v;
    int32_t ng;
};

struct BLds {
    float *Wk;
    uint32_t *Wi;
    VisCache vis;
    int32_t *Uid;
    float *Uk;
    int32_t *Ulo, *Urank, *Slo, *Ko, *Li;
    float *Tk;
};

__host__ __device__ inline int build_lds_bytes(int ef_cap, int vis_bits, int vis_kbits) {
    return ef_cap * 8 + (1 << vis_bits) * (vis_kbits ? 2 : 4) + kWave * 4 * 9;
}

__device__ inline BLds build_lds(char *p, const BuildArgs &A) {
    BLds L;
    L.Wk = reinterpret_cast<float *>(p);
    L.Wi = reinterpret_cast<uint32_t *>(L.Wk + A.ef_cap);
    L.vis.base = L.Wi + A.ef_cap;
    L.vis.bits = A.vis_bits;
    L.vis.kbits = A.vis_kbits;
    L.Uid = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(L.vis.base) +
                                        (1 << A.vis_bits) * (A.vis_kbits ? 2 : 4));
    L.Uk = reinterpret_cast<float *>(L.Uid + kWave);
    L.Ulo = reinterpret_cast<int32_t *>(L.Uk + kWave);
    L.Urank = L.Ulo + kWave;
    L.Slo = L.Urank + kWave;
    L.Ko = L.Slo + kWave;
    L.Li = L.Ko + kWave;
    L.Tk = reinterpret_cast<float *>(L.Li + kWave);
    return L;
}

// The neighbour list of v on layer l (width M0 on layer 0, M above).
__device__ __forceinline__ int32_t *layer_row(const BuildArgs &A, int32_t v, int l, int *width) {
    if (l == 0) {
        *width = A.M0;
        return A.adj0 + (int64_t)v * A.M0;
    }
    *width = A.M;
    return A.uadj + ((int64_t)A.upo[v] + (l - 1)) * A.M;
}

template <int NCH, int MET>
__device__ __forceinline__ void bdist(const BuildArgs &A, const int32_t *ids, int nrows, const float (&qv)[NCH][4],
                                      float *keys) {
    rows_base_dist<kBG, NCH, float, MET, 32>(A.base, A.pitch, ids, nrows, qv, keys, nullptr, A.metric_p);
}

// Best-first search of layer l from (ep, dep) with a list bounded by ef; the
// list ends ascending by (distance, id) in Wk / Wi (expanded bit set).
template <int NCH, int MET>
__device__ int search_layer(const BuildArgs &A, const BLds &L, const float (&qv)[NCH][4], int32_t ep, float dep,
                            int ef, int l) {
    const int lane = lane_id();
    L.vis.clear(lane);
    wave_sync();
    if (lane == 0) {
        L.Wk[0] = dep;
        L.Wi[0] = (uint32_t)ep;
        L.vis.mark_first(ep);
    }
    wave_sync();
    int nW = 1, lb = 0;
    for (int guard = 0; guard <= A.n; ++guard) {
        int pos = -1;
        uint32_t node = 0;
        for (int b0 = lb; b0 < nW; b0 += kWave) {
            const int i = b0 + lane;
            const uint64_t m = ballot(i < nW && !(L.Wi[i] & kExpBit));
            if (m) {
                pos = b0 + __ffsll((unsigned long long)m) - 1;
                node = L.Wi[pos];
                break;
            }
        }
        if (pos < 0) break;
        lb = pos;
        wave_sync();
        if (lane == 0) L.Wi[pos] = node | kExpBit;
        int width;
        const int32_t *row = layer_row(A, (int32_t)node, l, &width);
        const int32_t nb = lane < width ? row[lane] : -1;
        bool fresh = false;
        if (nb >= 0) {
            uint32_t vs, vt;
            L.vis.locate(nb, vs, vt);
            fresh = L.vis.test_and_mark(vs, vt);
        }
        wave_sync();
        const uint64_t fm = ballot(fresh);
        const int nnew = popc64(fm);
        if (nnew == 0) continue;
        if (fresh) L.Uid[lanes_below(fm)] = nb;
        wave_sync();
        bdist<NCH, MET>(A, L.Uid, nnew, qv, L.Uk);
        wave_sync();
        int min_new, n_in;
        nW = merge_into_sorted<true>(L.Wk, L.Wi, nW, ef, L.Uk, L.Uid, nnew, L.Ulo, L.Urank, L.Slo, false, &min_new,
                                     &n_in);
        if (min_new < lb) lb = min_new;
    }
    return nW;
}

// HNSW's neighbour selection by diversity: scan the candidates (ascending by
// distance to the base point, Ck / Ci) and keep e unless a kept r is closer
// to e than the base point is (dist(e, r) < Ck[e]); stop at msel kept. The
// kept ids land in Ko; returns their count.
template <int NCH, int MET>
__device__ int heuristic(const BuildArgs &A, const BLds &L, const float *Ck, const uint32_t *Ci, int nc, int msel) {
    const int lane = lane_id();
    int nk = 0;
    for (int i = 0; i < nc && nk < msel; ++i) {
        const int32_t e = (int32_t)(Ci[i] & kIdMask);
        const float de = Ck[i];
        bool good = true;
        if (nk > 0) {
            float qe[NCH][4];
            load_query<kBG, NCH>(A.base + (int64_t)e * A.pitch, A.d, qe);
            bdist<NCH, MET>(A, L.Ko, nk, qe, L.Tk);
            wave_sync();
            good = ballot(lane < nk && L.Tk[lane] < de) == 0;
        }
        if (good) {
            wave_sync();
            if (lane == 0) L.Ko[nk] = e;
            ++nk;
            wave_sync();
        }
    }
    return nk;
}

// One wave per batch member v = done + blockIdx.x: descent over the layers
// above its level, then per layer from min(level, lmax) down to 0 a search
// with efConstruction and the heuristic choice of M neighbours, written as
// v's own list on that layer and to the plan (for the reverse links).
template <int NCH, int MET>
__global__ void __launch_bounds__(64) build_plan_kernel(BuildArgs A) {
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const BLds L = build_lds(lds, A);
    const int i = blockIdx.x;
    if (i >= A.b) return;
    const int32_t v = (int32_t)(A.done + i);
    const int lane = lane_id();
    float qv[NCH][4];
    load_query<kBG, NCH>(A.base + (int64_t)v * A.pitch, A.d, qv);
    const int lv = A.level[v];
    int32_t cur = A.ep;
    if (lane == 0) L.Uid[0] = cur;
    wave_sync();
    bdist<NCH, MET>(A, L.Uid, 1, qv, L.Uk);
    wave_sync();
    float dcur = L.Uk[0];
    for (int l = A.lmax; l > lv; --l) {
        for (int guard = 0; guard <= A.n; ++guard) {
            wave_sync();
            int width;
            const int32_t *row = layer_row(A, cur, l, &width);
            const int32_t nb = lane < width ? row[lane] : -1;
            const int cnt = popc64(ballot(nb >= 0));
            if (nb >= 0) L.Uid[lane] = nb;  // valid ids come first in each list
            wave_sync();
            if (cnt == 0) break;
            bdist<NCH, MET>(A, L.Uid, cnt, qv, L.Uk);
            wave_sync();
            float kb = lane < cnt ? L.Uk[lane] : INFINITY;
            int32_t ib = lane < cnt ? L.Uid[lane] : 0x7fffffff;
            wave_argmin(kb, ib);
            if (!key_less(kb, (uint32_t)ib, dcur, (uint32_t)cur)) break;
            cur = ib;
            dcur = kb;
        }
    }
    const int top = lv < A.lmax ? lv : A.lmax;
    for (int l = top; l >= 0; --l) {
        wave_sync();
        const int nW = search_layer<NCH, MET>(A, L, qv, cur, dcur, A.efc, l);
        wave_sync();
        const int nk = heuristic<NCH, MET>(A, L, L.Wk, L.Wi, nW, A.M);
        int width;
        int32_t *row = layer_row(A, v, l, &width);
        const int32_t kept = lane < nk ? L.Ko[lane] : -1;
        if (lane < width) row[lane] = kept;
        if (lane < A.M) A.plan_ids[((int64_t)i * kBuildLayers + l) * A.M + lane] = kept;
        if (lane == 0) A.plan_cnt[i * kBuildLayers + l] = nk;
        cur = (int32_t)(L.Wi[0] & kIdMask);
        dcur = L.Wk[0];
    }
}

// One wave per reverse-link group (layer l, target u): u's list takes each
// requested source in order; a full list is re-selected from its entries and
// the new one, ascending by distance to u, with the same heuristic.
template <int NCH, int MET>
__global__ void __launch_bounds__(64) build_link_kernel(BuildArgs A) {
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const BLds L = build_lds(lds, A);
    const int g = blockIdx.x;
    if (g >= A.ng) return;
    const int l = A.g_l[g];
    const int32_t u = A.g_u[g];
    const int lane = lane_id();
    float qv[NCH][4];
    load_query<kBG, NCH>(A.base + (int64_t)u * A.pitch, A.d, qv);
    int width;
    int32_t *row = layer_row(A, u, l, &width);
    const int32_t id0 = lane < width ? row[lane] : -1;
    int cnt = popc64(ballot(id0 >= 0));
    L.Li[lane] = id0;
    wave_sync();
    for (int r = A.g_start[g]; r < A.g_start[g + 1]; ++r) {
        const int32_t v = A.req_v[r];
        wave_sync();
        if (lane == 0) L.Li[cnt] = v;  // cnt <= width < kWave
        wave_sync();
        if (cnt < width) {
            ++cnt;
            continue;
        }
        const int nc = cnt + 1;
        bdist<NCH, MET>(A, L.Li, nc, qv, L.Uk);
        wave_sync();
        if (lane < nc) {  // ascending (distance to u, id)
            const float kk = L.Uk[lane];
            const uint32_t ii = (uint32_t)L.Li[lane];
            int rank = 0;
            for (int j = 0; j < nc; ++j) rank += key_less(L.Uk[j], (uint32_t)L.Li[j], kk, ii) ? 1 : 0;
            L.Wk[rank] = kk;
            L.Wi[rank] = ii;
        }
        wave_sync();
        const int nk = heuristic<NCH, MET>(A, L, L.Wk, L.Wi, nc, width);
        wave_sync();
        L.Li[lane] = lane < nk ? L.Ko[lane] : -1;
        cnt = nk;
    }
    wave_sync();
    if (lane < width) row[lane] = L.Li[lane];
}

#define UHNSW_BUILD_NCH_SWITCH(nch, MACRO) \
    switch (nch) {                         \
        case 1: MACRO(1); break;           \
        case 2: MACRO(2); break;           \
        case 4: MACRO(4); break;           \
        default: MACRO(16); break;         \
    }

template <int MET>
hipError_t launch_plan_met(const BuildArgs &a, int nch, hipStream_t s) {
#define P_L(N) hipLaunchKernelGGL((build_plan_kernel<N, MET>), dim3(a.b), dim3(kWave), a.lds_wave_bytes, s, a);
    UHNSW_BUILD_NCH_SWITCH(nch, P_L)
#undef P_L
    return hipGetLastError();
}

template <int MET>
hipError_t launch_link_met(const BuildArgs &a, int nch, hipStream_t s) {
#define K_L(N) hipLaunchKernelGGL((build_link_kernel<N, MET>), dim3(a.ng), dim3(kWave), a.lds_wave_bytes, s, a);
    UHNSW_BUILD_NCH_SWITCH(nch, K_L)
#undef K_L
    return hipGetLastError();
}

hipError_t launch_plan(const BuildArgs &a, int metric, int nch, hipStream_t s) {
    return metric == 1   ? launch_plan_met<kMetL1>(a, nch, s)
           : metric == 2 ? launch_plan_met<kMetL2>(a, nch, s)
           : metric == 3 ? launch_plan_met<kMetL05>(a, nch, s)
                         : launch_plan_met<kMetLp>(a, nch, s);
}

hipError_t launch_link(const BuildArgs &a, int metric, int nch, hipStream_t s) {
    return metric == 1   ? launch_link_met<kMetL1>(a, nch, s)
           : metric == 2 ? launch_link_met<kMetL2>(a, nch, s)
           : metric == 3 ? launch_link_met<kMetL05>(a, nch, s)
                         : launch_link_met<kMetLp>(a, nch, s);
}

uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

struct Req {
    int32_t l, u, v;
};

// Device buffers of one build, released on every exit path.
struct DevMem {
    std::vector<void *> ptrs;
    ~DevMem() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    hipError_t alloc(T **p, size_t count) {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) ptrs.push_back(q);
        *p = static_cast<T *>(q);
        return e;
    }
};

struct HostPinned {
    std::vector<void *> ptrs;
    ~HostPinned() {
        for (void *p : ptrs) (void)hipHostFree(p);
    }
    template <typename T>
    hipError_t alloc(T **p, size_t count) {
        void *q = nullptr;
        hipError_t e = hipHostMalloc(&q, std::max<size_t>(count, 1) * sizeof(T), hipHostMallocDefault);
        if (e == hipSuccess) ptrs.push_back(q);
        *p = static_cast<T *>(q);
        return e;
    }
};

}  // namespace
}  // namespace uhnsw

using namespace uhnsw;

struct uhnsw_built_graph {
    int64_t n = 0;
    int32_t M = 0, max_level = 0, entry = 0;
    double seconds = 0.0;
    int64_t batches = 0;
    std::vector<int8_t> level;
    std::vector<std::vector<int64_t>> row_ptr;
    std::vector<std::vector<int32_t>> col, nodes;
};

extern "C" {

static int build_graph_body(uhnsw_ctx *ctx, const float *base, int64_t n, int32_t d, int32_t metric, float metric_p,
                            int32_t M, int32_t ef_construction, uint64_t seed, int32_t batch_max,
                            uhnsw_built_graph **out) {
    if (!ctx) return UHNSW_EINVAL;
    auto build_fail = [ctx](int code, const std::string &msg) {
        ctx_set_error(ctx, ("uhnsw_build_graph: " + msg).c_str());
        return code;
    };
    if (!base || !out) return build_fail(UHNSW_EINVAL, "NULL argument");
    *out = nullptr;
    if (n < 1 || n > INT32_MAX) return build_fail(UHNSW_EINVAL, "n outside [1, 2^31)");
    if (d < 1 || d > UHNSW_DMAX) return build_fail(UHNSW_EINVAL, "d outside [1, UHNSW_DMAX]");
    if (metric < 1 || metric > 4)
        return build_fail(UHNSW_EINVAL, "metric must be 1 (L1), 2 (L2), 3 (L0.5) or 4 (L_p)");
    if (metric == 4 && !(metric_p >= 0.2f && metric_p <= 2.0f))
        return build_fail(UHNSW_EINVAL, "metric_p outside [0.2, 2]");
    if (M < 2 || 2 * M >= kWave) return build_fail(UHNSW_EINVAL, "M outside [2, 31]");
    if (ef_construction < 1 || ef_construction > UHNSW_EFMAX)
        return build_fail(UHNSW_EINVAL, "ef_construction outside [1, UHNSW_EFMAX]");
    if (batch_max < 1 || batch_max > (1 << 16)) return build_fail(UHNSW_EINVAL, "batch_max outside [1, 65536]");
    for (int64_t i = 0; i < n * (int64_t)d; ++i)
        if (!std::isfinite(base[i])) return build_fail(UHNSW_EINVAL, "a base value is not finite");
    const auto t0 = std::chrono::steady_clock::now();
    const int dev = ctx_device(ctx);
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return build_fail(UHNSW_EDEVICE, hipGetErrorString(e));
    const int nch = d <= 64 ? 1 : d <= 128 ? 2 : d <= 256 ? 4 : 16;
    const int64_t pitch = (int64_t)nch * kBG * 4;
    const int M0 = 2 * M;
    // levels and upper-layer rows (host: the same draw as the CPU builder)
    auto G = std::make_unique<uhnsw_built_graph>();
    G->n = n;
    G->M = M;
    G->level.resize((size_t)n);
    std::vector<int32_t> upo((size_t)n, -1);
    const double ml = 1.0 / std::log((double)M);
    int64_t rows = 0;
    for (int64_t v = 0; v < n; ++v) {
        const uint64_t z = splitmix64(seed ^ ((uint64_t)v * 0x9E3779B97F4A7C15ULL));
        const double uu = ((double)(z >> 11) + 1.0) * (1.0 / 9007199254740992.0);  // (0, 1]
        int lv = (int)std::floor(-std::log(uu) * ml);
        if (lv > kLevelCap) lv = kLevelCap;
        G->level[(size_t)v] = (int8_t)lv;
        if (lv) {
            upo[(size_t)v] = (int32_t)rows;
            rows += lv;
        }
        if (rows * M >= INT32_MAX) return build_fail(UHNSW_EUNSUPPORTED, "upper layers too large");
    }
    // visited cache: as many slots as keep a wave within 24 KiB of LDS
    const int ef_cap = (std::max(ef_construction, kWave) + 3) / 4 * 4;
    int vis_bits = 13, vis_kbits = 0;
    for (; vis_bits >= 10; --vis_bits) {
        int kb = 1;
        while (kb < 31 && ((int64_t)1 << kb) < n) ++kb;
        if (kb < vis_bits + 1) kb = vis_bits + 1;
        vis_kbits = vis_tags_fit(kb, vis_bits) ? kb : 0;
        if (build_lds_bytes(ef_cap, vis_bits, vis_kbits) <= 24 * 1024) break;
    }
    if (vis_bits < 10) return build_fail(UHNSW_EUNSUPPORTED, "ef_construction too large for the LDS plan");
    hipStream_t s = nullptr;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
        return build_fail(UHNSW_EDEVICE, hipGetErrorString(e));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    } sg{s};
    DevMem dm;
    HostPinned hm;
    BuildArgs a{};
    float *d_base = nullptr;
    int32_t *d_adj0 = nullptr, *d_uadj = nullptr, *d_upo = nullptr, *d_plan = nullptr, *d_pcnt = nullptr;
    int32_t *d_gl = nullptr, *d_gu = nullptr, *d_gs = nullptr, *d_rv = nullptr;
    int8_t *d_level = nullptr;
    const size_t plan_ints = (size_t)batch_max * kBuildLayers * M;
    const size_t req_max = plan_ints;
    int32_t *h_plan = nullptr, *h_pcnt = nullptr, *h_grp = nullptr;
#define B_TRY(call)                                                                 \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            return build_fail(e_ == hipErrorOutOfMemory ? UHNSW_ENOMEM : UHNSW_EDEVICE, \
                              std::string(#call ": ") + hipGetErrorString(e_));     \
    } while (0)
    B_TRY(dm.alloc(&d_base, (size_t)n * pitch));
    B_TRY(dm.alloc(&d_adj0, (size_t)n * M0));
    B_TRY(dm.alloc(&d_uadj, (size_t)std::max<int64_t>(rows, 1) * M));
    B_TRY(dm.alloc(&d_upo, (size_t)n));
    B_TRY(dm.alloc(&d_level, (size_t)n));
    B_TRY(dm.alloc(&d_plan, plan_ints));
    B_TRY(dm.alloc(&d_pcnt, (size_t)batch_max * kBuildLayers));
    B_TRY(dm.alloc(&d_gl, req_max));
    B_TRY(dm.alloc(&d_gu, req_max));
    B_TRY(dm.alloc(&d_gs, req_max + 1));
    B_TRY(dm.alloc(&d_rv, req_max));
    B_TRY(hm.alloc(&h_plan, plan_ints));
    B_TRY(hm.alloc(&h_pcnt, (size_t)batch_max * kBuildLayers));
    B_TRY(hm.alloc(&h_grp, 4 * req_max + 1));
    {
        // rows zero padded to the pitch, uploaded in slices
        const int64_t slice = std::max<int64_t>(1, ((int64_t)64 << 20) / (pitch * 4));
        std::vector<float> buf((size_t)std::min(slice, n) * pitch, 0.0f);
        for (int64_t r0 = 0; r0 < n; r0 += slice) {
            const int64_t nr = std::min(slice, n - r0);
            for (int64_t r = 0; r < nr; ++r)
                std::memcpy(&buf[(size_t)r * pitch], base + (r0 + r) * d, sizeof(float) * d);
            B_TRY(hipMemcpy(d_base + r0 * pitch, buf.data(), sizeof(float) * nr * pitch, hipMemcpyHostToDevice));
        }
    }
    B_TRY(hipMemcpy(d_upo, upo.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    B_TRY(hipMemcpy(d_level, G->level.data(), (size_t)n, hipMemcpyHostToDevice));
    B_TRY(launch_fill_i32(d_adj0, -1, n * M0, s));
    B_TRY(launch_fill_i32(d_uadj, -1, std::max<int64_t>(rows, 1) * M, s));
    a.base = d_base;
    a.pitch = pitch;
    a.n = n;
    a.d = d;
    a.adj0 = d_adj0;
    a.uadj = d_uadj;
    a.upo = d_upo;
    a.level = d_level;
    a.M = M;
    a.M0 = M0;
    a.efc = ef_construction;
    a.metric_p = metric == 4 ? metric_p : 0.0f;
    a.ef_cap = ef_cap;
    a.vis_bits = vis_bits;
    a.vis_kbits = vis_kbits;
    a.lds_wave_bytes = build_lds_bytes(ef_cap, vis_bits, vis_kbits);
    a.plan_ids = d_plan;
    a.plan_cnt = d_pcnt;
    a.g_l = d_gl;
    a.g_u = d_gu;
    a.g_start = d_gs;
    a.req_v = d_rv;

    int32_t entry = 0;
    int max_level = G->level[0];
    int64_t done = 1;
    std::vector<Req> reqs;
    reqs.reserve(req_max);
    while (done < n) {
        int64_t b = std::min<int64_t>(std::max<int64_t>(done / 64, 1), batch_max);
        b = std::min<int64_t>(b, n - done);
        a.done = done;
        a.b = (int32_t)b;
        a.lmax = max_level;
        a.ep = entry;
        B_TRY(launch_plan(a, metric, nch, s));
        B_TRY(hipMemcpyAsync(h_pcnt, d_pcnt, sizeof(int32_t) * b * kBuildLayers, hipMemcpyDeviceToHost, s));
        B_TRY(hipMemcpyAsync(h_plan, d_plan, sizeof(int32_t) * b * kBuildLayers * M, hipMemcpyDeviceToHost, s));
        B_TRY(hipStreamSynchronize(s));
        // reverse-link requests (layer, target, source), grouped by (layer,
        // target), each group's sources ascending
        reqs.clear();
        for (int64_t i = 0; i < b; ++i) {
            const int32_t v = (int32_t)(done + i);
            const int top = std::min<int>(G->level[(size_t)v], max_level);
            for (int l = 0; l <= top; ++l) {
                const int c = h_pcnt[i * kBuildLayers + l];
                for (int j = 0; j < c; ++j) reqs.push_back({l, h_plan[(i * kBuildLayers + l) * M + j], v});
            }
        }
        std::sort(reqs.begin(), reqs.end(), [](const Req &x, const Req &y) {
            return x.l != y.l ? x.l < y.l : x.u != y.u ? x.u < y.u : x.v < y.v;
        });
        int32_t *gl = h_grp, *gu = h_grp + req_max, *gs = h_grp + 2 * req_max, *rv = h_grp + 3 * req_max + 1;
        int32_t ng = 0;
        for (size_t r = 0; r < reqs.size(); ++r) {
            if (r == 0 || reqs[r].l != reqs[r - 1].l || reqs[r].u != reqs[r - 1].u) {
                gl[ng] = reqs[r].l;
                gu[ng] = reqs[r].u;
                gs[ng] = (int32_t)r;
                ++ng;
            }
            rv[r] = reqs[r].v;
        }
        gs[ng] = (int32_t)reqs.size();
        if (ng > 0) {
            B_TRY(hipMemcpyAsync(d_gl, gl, sizeof(int32_t) * ng, hipMemcpyHostToDevice, s));
            B_TRY(hipMemcpyAsync(d_gu, gu, sizeof(int32_t) * ng, hipMemcpyHostToDevice, s));
            B_TRY(hipMemcpyAsync(d_gs, gs, sizeof(int32_t) * (ng + 1), hipMemcpyHostToDevice, s));
            B_TRY(hipMemcpyAsync(d_rv, rv, sizeof(int32_t) * reqs.size(), hipMemcpyHostToDevice, s));
            a.ng = ng;
            B_TRY(launch_link(a, metric, nch, s));
            // the pinned request arrays are rewritten by the next batch
            B_TRY(hipStreamSynchronize(s));
        }
        for (int64_t i = 0; i < b; ++i) {
            const int32_t v = (int32_t)(done + i);
            if (G->level[(size_t)v] > max_level) {
                max_level = G->level[(size_t)v];
                entry = v;
            }
        }
        done += b;
        ++G->batches;
    }
    B_TRY(hipStreamSynchronize(s));
    // per-layer CSR: nodes ascending, each list's valid prefix
    std::vector<int32_t> adj0((size_t)n * M0), uadj((size_t)std::max<int64_t>(rows, 1) * M);
    B_TRY(hipMemcpy(adj0.data(), d_adj0, sizeof(int32_t) * adj0.size(), hipMemcpyDeviceToHost));
    B_TRY(hipMemcpy(uadj.data(), d_uadj, sizeof(int32_t) * uadj.size(), hipMemcpyDeviceToHost));
#undef B_TRY
    G->max_level = max_level;
    G->entry = entry;
    G->row_ptr.resize(max_level + 1);
    G->col.resize(max_level + 1);
    G->nodes.resize(max_level + 1);
    for (int l = 0; l <= max_level; ++l) {
        auto &rp = G->row_ptr[l];
        auto &col = G->col[l];
        rp.push_back(0);
        for (int64_t v = 0; v < n; ++v) {
            if (G->level[(size_t)v] < l) continue;
            const int32_t *lst = l == 0 ? &adj0[(size_t)v * M0] : &uadj[((size_t)upo[(size_t)v] + (l - 1)) * M];
            const int w = l == 0 ? M0 : M;
            for (int j = 0; j < w && lst[j] >= 0; ++j) col.push_back(lst[j]);
            rp.push_back((int64_t)col.size());
            if (l > 0) G->nodes[l].push_back((int32_t)v);
        }
        if (col.empty()) col.push_back(0);  // a valid pointer for empty layers
        if (l > 0 && G->nodes[l].empty()) G->nodes[l].push_back(0);
    }
    G->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = G.release();
    return UHNSW_OK;
}

int uhnsw_build_graph(uhnsw_ctx *ctx, const float *base, int64_t n, int32_t d, int32_t metric, float metric_p,
                      int32_t M, int32_t ef_construction, uint64_t seed, int32_t batch_max,
                      uhnsw_built_graph **out) {
    const auto body = [&] {
        return build_graph_body(ctx, base, n, d, metric, metric_p, M, ef_construction, seed, batch_max, out);
    };
    return no_throw("uhnsw_build_graph", body, [&](const char *w) { if (ctx) ctx_set_error(ctx, w); });
}

int uhnsw_built_graph_view(const uhnsw_built_graph *g, uhnsw_graph *out, double *build_seconds,
                           int64_t *batches) {
    if (!g || !out) return UHNSW_EINVAL;
    std::memset(out, 0, sizeof *out);
    out->M = g->M;
    out->max_level = g->max_level;
    out->entry_point = g->entry;
    out->level = g->level.data();
    for (int l = 0; l <= g->max_level; ++l) {
        out->n_nodes[l] = l == 0 ? g->n : (int64_t)g->row_ptr[l].size() - 1;
        out->nodes[l] = l == 0 ? nullptr : g->nodes[l].data();
        out->row_ptr[l] = g->row_ptr[l].data();
        out->col[l] = g->col[l].data();
    }
    if (build_seconds) *build_seconds = g->seconds;
    if (batches) *batches = g->batches;
    return UHNSW_OK;
}

void uhnsw_built_graph_free(uhnsw_built_graph *g) { delete g; }

}  // extern "C"
