// gfx950 kernels of the U-HNSW query path (U-HNSW paper, Sec. 3.1 and
// Algorithm 1): the verification kernel of the two-kernel form, the cost-
// ordering pre-pass kernels, the utility kernels and the launchers. The
// walk, fused and descent kernels are instantiated per (storage, index
// variant) in uhnsw_walk_part.hip; all device code is in uhnsw_device.h.
#include <mutex>

#include "uhnsw_device.h"

namespace uhnsw {

// ------------------------------------------------ fixed scratch region
// The scratch of uhnsw_search_device_noalloc: one region per device,
// reserved when the code object loads and held until the process ends.
// Host code must not use the array's name as an address (it is a host-side
// stand-in); noalloc_scratch returns the device address, looked up once per
// device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(int device, void **out) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

// One workgroup: per graph the sum and count of entry distances, and the
// sum and count of ef, over all searchable queries (fixed order, no atomics).
__global__ void __launch_bounds__(256) order_mean_kernel(SearchArgs A, OrderArgs O) {
    __shared__ float part[6][256 / kWave];
    float v[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t qi = threadIdx.x; qi < A.nq; qi += blockDim.x) {
        const float dist = O.dist[qi];
        if (dist < 0.0f) continue;
        const int gsel = (A.p[qi] <= A.cutoff) ? 0 : 1;
        v[2 * gsel] += dist;
        v[2 * gsel + 1] += 1.0f;
        v[4] += (float)A.ef[qi];
        v[5] += 1.0f;
    }
    const int wave = threadIdx.x / kWave, lane = lane_id();
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        float x = v[j];
#pragma unroll
        for (int o = kWave / 2; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
        if (lane == 0) part[j][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        float x = 0.0f;
        for (int w = 0; w < (int)blockDim.x / kWave; ++w) x += part[threadIdx.x][w];
        O.gsum[threadIdx.x] = x;
    }
}

// Bucket of a query: predicted length r (entry distance over its graph's
// mean times ef over the mean ef) on a log scale, 16 buckets per doubling
// over [1/4, 4), largest first; unsearchable queries go to the last bucket.
__device__ __forceinline__ int order_bucket(const OrderArgs &O, const SearchArgs &A, int64_t qi) {
    const float dist = O.dist[qi];
    if (dist < 0.0f) return kOrderBuckets - 1;
    const int gsel = (A.p[qi] <= A.cutoff) ? 0 : 1;
    const float mean = O.gsum[2 * gsel] / fmaxf(O.gsum[2 * gsel + 1], 1.0f);
    const float mean_ef = O.gsum[4] / fmaxf(O.gsum[5], 1.0f);
    const float r = (mean > 0.0f ? dist / mean : 1.0f) * (mean_ef > 0.0f ? (float)A.ef[qi] / mean_ef : 1.0f);
    int b = r > 0.0f ? (int)floorf(log2f(r) * 16.0f) + 32 : 0;
    b = b < 0 ? 0 : (b > kOrderBuckets - 2 ? kOrderBuckets - 2 : b);
    return kOrderBuckets - 2 - b;
}

// Counts per bucket: a workgroup histogram in LDS, then one global add per
// non-empty bucket and workgroup.
__global__ void __launch_bounds__(256) order_count_kernel(SearchArgs A, OrderArgs O) {
    __shared__ int h[kOrderBuckets];
    if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (qi < A.nq) atomicAdd(&h[order_bucket(O, A, qi)], 1);
    __syncthreads();
    if (threadIdx.x < kOrderBuckets && h[threadIdx.x] > 0) atomicAdd(&O.bcnt[threadIdx.x], h[threadIdx.x]);
}

// One wave: exclusive prefix sum of the bucket counts into the cursors.
__global__ void order_scan_kernel(OrderArgs O) {
    const int lane = lane_id();
    int v = lane < kOrderBuckets ? O.bcnt[lane] : 0;
    int incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
    }
    if (lane < kOrderBuckets) O.bcnt[kOrderBuckets + lane] = incl - v;
}

// Positions: each workgroup reserves one range per non-empty bucket from the
// global cursors and hands out places inside it through LDS counters.
__global__ void __launch_bounds__(256) order_scatter_kernel(SearchArgs A, OrderArgs O) {
    __shared__ int h[kOrderBuckets];
    __shared__ int base[kOrderBuckets];
    if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = qi < A.nq ? order_bucket(O, A, qi) : 0;
    if (qi < A.nq) atomicAdd(&h[b], 1);
    __syncthreads();
    if (threadIdx.x < kOrderBuckets) {
        const int c = h[threadIdx.x];
        base[threadIdx.x] = c > 0 ? atomicAdd(&O.bcnt[kOrderBuckets + threadIdx.x], c) : 0;
        h[threadIdx.x] = 0;
    }
    __syncthreads();
    if (qi < A.nq) O.order[base[b] + atomicAdd(&h[b], 1)] = (int32_t)qi;
}

__global__ void fill_i32_kernel(int32_t *dst, int32_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = v;
}

// FP32 -> bfloat16 / binary16, round to nearest even.
__global__ void convert_kernel(const float *src, uint16_t *dst, int64_t count, int storage) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float f = src[i];
    if (storage == UHNSW_STORE_BF16) {
        const uint32_t u = __float_as_uint(f);
        if ((u & 0x7fffffffu) > 0x7f800000u) {
            dst[i] = (uint16_t)((u >> 16) | 0x40u);
        } else {
            const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
            dst[i] = (uint16_t)(r >> 16);
        }
    } else {
        dst[i] = __half_as_ushort(__float2half_rn(f));
    }
}

// ---------------------------------------------------------------- launch
// The per-(storage, variant) instantiations of uhnsw_walk_part.hip.
#define UHNSW_PART_FNS(S, E)                                                                             \
    hipError_t launch_walk_##S##_##E(const SearchArgs &, int, int, hipStream_t);                         \
    hipError_t launch_search_##S##_##E(const SearchArgs &, int, int, hipStream_t);                       \
    hipError_t launch_descend_##S##_##E(const SearchArgs &, const OrderArgs &, int, int, int, hipStream_t); \
    const void *walk_stub_##S##_##E(int);                                                                \
    const void *search_stub_##S##_##E(int, int);
UHNSW_PART_FNS(0, 0)
UHNSW_PART_FNS(1, 0)
UHNSW_PART_FNS(2, 0)
UHNSW_PART_FNS(0, 1)
UHNSW_PART_FNS(1, 1)
UHNSW_PART_FNS(2, 1)
#undef UHNSW_PART_FNS

namespace {
struct PartFns {
    hipError_t (*walk)(const SearchArgs &, int, int, hipStream_t);
    hipError_t (*search)(const SearchArgs &, int, int, hipStream_t);
    hipError_t (*descend)(const SearchArgs &, const OrderArgs &, int, int, int, hipStream_t);
    const void *(*walk_stub)(int);
    const void *(*search_stub)(int, int);
};
#define UHNSW_PART_ROW(S, E) \
    { launch_walk_##S##_##E, launch_search_##S##_##E, launch_descend_##S##_##E, walk_stub_##S##_##E, search_stub_##S##_##E }
// [storage][variant]
const PartFns kParts[3][2] = {{UHNSW_PART_ROW(0, 0), UHNSW_PART_ROW(0, 1)},
                              {UHNSW_PART_ROW(1, 0), UHNSW_PART_ROW(1, 1)},
                              {UHNSW_PART_ROW(2, 0), UHNSW_PART_ROW(2, 1)}};
#undef UHNSW_PART_ROW

const PartFns *part_of(int storage, bool ext) {
    if (storage < UHNSW_STORE_F32 || storage > UHNSW_STORE_F16) return nullptr;
    return &kParts[storage][ext ? 1 : 0];
}
}  // namespace

hipError_t launch_walk(const SearchArgs &a, int layout, int grid, hipStream_t s) {
    const PartFns *f = part_of(a.storage, a.ext != 0);
    return f ? f->walk(a, layout, grid, s) : hipErrorInvalidValue;
}

hipError_t launch_verify(const SearchArgs &a, int layout, int grid, hipStream_t s) {
    const dim3 blk(a.waves_per_block * kWave);
    const size_t lds = (size_t)a.lds_wave_bytes * a.waves_per_block;
#define V_LAUNCH(G, NCH) hipLaunchKernelGGL((verify_kernel<G, NCH>), dim3(grid), blk, lds, s, a);
    UHNSW_LAYOUT_SWITCH(layout, V_LAUNCH)
#undef V_LAUNCH
    return hipGetLastError();
}

hipError_t launch_search(const SearchArgs &a, int layout, int grid, hipStream_t s) {
    const PartFns *f = part_of(a.storage, a.ext != 0);
    return f ? f->search(a, layout, grid, s) : hipErrorInvalidValue;
}

hipError_t launch_order(const SearchArgs &a, const OrderArgs &o, int layout, hipStream_t s) {
    const int wpb = 4;
    const int grid = (int)((a.nq + wpb - 1) / wpb);
    SearchArgs b = a;
    b.waves_per_block = wpb;
    const PartFns *f = part_of(a.storage, a.ext != 0);
    if (!f) return hipErrorInvalidValue;
    hipError_t e = f->descend(b, o, layout, grid, wpb, s);
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)((a.nq + 255) / 256);
    hipLaunchKernelGGL(order_mean_kernel, dim3(1), dim3(256), 0, s, a, o);
    hipLaunchKernelGGL(order_count_kernel, dim3(blocks), dim3(256), 0, s, a, o);
    hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(kWave), 0, s, o);
    hipLaunchKernelGGL(order_scatter_kernel, dim3(blocks), dim3(256), 0, s, a, o);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *dst, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dst, v, n);
    return hipGetLastError();
}

hipError_t launch_convert(const float *src, void *dst, int64_t count, int storage, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(convert_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src,
                       reinterpret_cast<uint16_t *>(dst), count, storage);
    return hipGetLastError();
}

int walk_lds_bytes(int ef_cap, int vis_bits, int vis_kbits, bool ext) {
    return walk_lds_bytes_impl(ef_cap, vis_bits, vis_kbits, ext);
}
int verify_lds_bytes(int kv_cap) { return verify_lds_bytes_impl(kv_cap); }

// Host stubs of the walk and fused kernels by row layout, storage, beam width
// and index variant (for occupancy queries).
const void *walk_kernel_ptr(int layout, int storage, bool ext) {
    const PartFns *f = part_of(storage, ext);
    return f ? f->walk_stub(layout) : nullptr;
}

const void *search_kernel_ptr(int layout, int storage, int beam, bool ext) {
    const PartFns *f = part_of(storage, ext);
    return f ? f->search_stub(layout, beam) : nullptr;
}

const void *verify_kernel_ptr(int layout) {
    switch (layout) {
        case L8x4x1: return reinterpret_cast<const void *>(&verify_kernel<8, 1>);
        case L8x4x2: return reinterpret_cast<const void *>(&verify_kernel<8, 2>);
        case L8x4x4: return reinterpret_cast<const void *>(&verify_kernel<8, 4>);
        case L16x4x4: return reinterpret_cast<const void *>(&verify_kernel<16, 4>);
        case L32x4x4: return reinterpret_cast<const void *>(&verify_kernel<32, 4>);
        default: return reinterpret_cast<const void *>(&verify_kernel<64, 4>);
    }
}

}  // namespace uhnsw
