// Ceiling probes for reading the rooflines of the query path's kernels:
// measurement only, not called by any search.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "uhnsw_internal.h"

namespace uhnsw {

// Random row gathers with the walk's lane mapping (8 lanes per row, 16-B
// loads, 32 rows in flight per wave) but no dependency between batches: the
// rate HBM sustains for this access pattern, the ceiling the walk works
// under. Each wave draws its row ids from a hash of (wave, batch, row).
__device__ __forceinline__ uint32_t probe_hash(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

template <int NCH>
__global__ void __launch_bounds__(256) gather_probe_kernel(const float4 *__restrict__ base, int64_t n,
                                                           int pitch_vec4, int iters, uint32_t seed, float *sink) {
    constexpr int RB = 4;
    const int lane = (int)__lane_id();
    const int grp = lane / 8, gl = lane % 8;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    float acc = 0.0f;
    for (int it = 0; it < iters; ++it) {
        float4 v[RB][NCH];
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const uint32_t h = probe_hash(seed ^ probe_hash(wave * 0x9E3779B9u + (uint32_t)it * 64u + b * 8 + grp));
            const int64_t row = (int64_t)(h % (uint32_t)n);
#pragma unroll
            for (int c = 0; c < NCH; ++c) v[b][c] = base[row * pitch_vec4 + c * 8 + gl];
        }
#pragma unroll
        for (int b = 0; b < RB; ++b)
#pragma unroll
            for (int c = 0; c < NCH; ++c) acc += (v[b][c].x + v[b][c].y) + (v[b][c].z + v[b][c].w);
    }
    if (acc == 1.2345e-30f) sink[0] = acc;  // keeps the loads; practically never taken
}

// Independent chains of v_log_f32 -> v_mul -> v_exp_f32 (x <- x^0.999 stays in
// (0, 2]): the issue rate of the transcendental unit.
__global__ void __launch_bounds__(256) trans_probe_kernel(int iters, float *sink) {
    constexpr int CH = 8;
    float x[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) x[j] = 1.0f + 1e-3f * (float)((threadIdx.x + j) % 512);
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int j = 0; j < CH; ++j) x[j] = __builtin_amdgcn_exp2f(0.999f * __builtin_amdgcn_logf(x[j]));
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < CH; ++j) acc += x[j];
    if (acc == 1.2345e-30f) sink[0] = acc;
}

hipError_t launch_gather_probe(const float *base, int64_t n, int64_t pitch, int row_bytes, int blocks, int iters,
                               uint32_t seed, float *sink, hipStream_t s) {
    const auto *b4 = reinterpret_cast<const float4 *>(base);
    const int pv = (int)(pitch / 4);
    switch (row_bytes) {
        case 128: hipLaunchKernelGGL(gather_probe_kernel<1>, dim3(blocks), dim3(256), 0, s, b4, n, pv, iters, seed, sink); break;
        case 256: hipLaunchKernelGGL(gather_probe_kernel<2>, dim3(blocks), dim3(256), 0, s, b4, n, pv, iters, seed, sink); break;
        case 512: hipLaunchKernelGGL(gather_probe_kernel<4>, dim3(blocks), dim3(256), 0, s, b4, n, pv, iters, seed, sink); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_trans_probe(int blocks, int iters, float *sink, hipStream_t s) {
    hipLaunchKernelGGL(trans_probe_kernel, dim3(blocks), dim3(256), 0, s, iters, sink);
    return hipGetLastError();
}

}  // namespace uhnsw
