// The walk, fused walk + verification and descent kernels for one walk
// storage type and one index variant. This file is compiled once per
// (UHNSW_PART_S, UHNSW_PART_E): S = 0 FP32, 1 BF16, 2 FP16 rows; E = 0 the
// (G1, G2) pair of Sec. 3.1, 1 the (G_0.5, G_1) pair of Sec. 4.5. Each
// compilation defines launch_*_S_E and *_stub_S_E, which the dispatchers of
// uhnsw_kernels.hip call.
#include "uhnsw_device.h"

#if !defined(UHNSW_PART_S) || !defined(UHNSW_PART_E)
#error "compile with -DUHNSW_PART_S=0|1|2 -DUHNSW_PART_E=0|1"
#endif

namespace uhnsw {

namespace {
template <int S>
struct PartType;
template <>
struct PartType<0> {
    using T = float;
};
template <>
struct PartType<1> {
    using T = bf16_t;
};
template <>
struct PartType<2> {
    using T = f16_t;
};
using PT = PartType<UHNSW_PART_S>::T;
constexpr bool PE = UHNSW_PART_E != 0;
}  // namespace

#define UHNSW_CAT5(a, b, c, d, e) a##b##c##d##e
#define UHNSW_XCAT5(a, b, c, d, e) UHNSW_CAT5(a, b, c, d, e)
#define UHNSW_PFN(fn) UHNSW_XCAT5(fn, _, UHNSW_PART_S, _, UHNSW_PART_E)

hipError_t UHNSW_PFN(launch_walk)(const SearchArgs &a, int layout, int grid, hipStream_t s) {
    const dim3 blk(a.waves_per_block * kWave);
    const size_t lds = (size_t)a.lds_wave_bytes * a.waves_per_block;
#define W_LAUNCH(G, NCH) hipLaunchKernelGGL((walk_kernel<G, NCH, PT, PE>), dim3(grid), blk, lds, s, a);
    UHNSW_LAYOUT_SWITCH(layout, W_LAUNCH)
#undef W_LAUNCH
    return hipGetLastError();
}

hipError_t UHNSW_PFN(launch_search)(const SearchArgs &a, int layout, int grid, hipStream_t s) {
    const dim3 blk(a.waves_per_block * kWave);
    const size_t lds = (size_t)a.lds_wave_bytes * a.waves_per_block;
#define S_LAUNCH(G, NCH)                                                                         \
    if (a.beam == 2)                                                                             \
        hipLaunchKernelGGL((search_kernel<G, NCH, PT, 2, PE>), dim3(grid), blk, lds, s, a);      \
    else                                                                                         \
        hipLaunchKernelGGL((search_kernel<G, NCH, PT, 1, PE>), dim3(grid), blk, lds, s, a);
    UHNSW_LAYOUT_SWITCH(layout, S_LAUNCH)
#undef S_LAUNCH
    return hipGetLastError();
}

// descent pre-pass: `grid` blocks of `wpb` waves, one query per wave
hipError_t UHNSW_PFN(launch_descend)(const SearchArgs &b, const OrderArgs &o, int layout, int grid, int wpb,
                                     hipStream_t s) {
    const size_t lds = (size_t)wpb * descend_lds_wave_bytes(PE);
#define D_LAUNCH(G, NCH) \
    hipLaunchKernelGGL((descend_kernel<G, NCH, PT, PE>), dim3(grid), dim3(wpb * kWave), lds, s, b, o);
    UHNSW_LAYOUT_SWITCH(layout, D_LAUNCH)
#undef D_LAUNCH
    return hipGetLastError();
}

// Host stubs by row layout (for occupancy queries).
const void *UHNSW_PFN(walk_stub)(int layout) {
#define WB(G, NCH) return reinterpret_cast<const void *>(&walk_kernel<G, NCH, PT, PE>);
    switch (layout) {
        case L8x4x1: WB(8, 1)
        case L8x4x2: WB(8, 2)
        case L8x4x4: WB(8, 4)
        case L16x4x4: WB(16, 4)
        case L32x4x4: WB(32, 4)
        default: WB(64, 4)
    }
#undef WB
}

const void *UHNSW_PFN(search_stub)(int layout, int beam) {
#define SB(G, NCH)                                                                          \
    return beam == 2 ? reinterpret_cast<const void *>(&search_kernel<G, NCH, PT, 2, PE>) \
                     : reinterpret_cast<const void *>(&search_kernel<G, NCH, PT, 1, PE>);
    switch (layout) {
        case L8x4x1: SB(8, 1)
        case L8x4x2: SB(8, 2)
        case L8x4x4: SB(8, 4)
        case L16x4x4: SB(16, 4)
        case L32x4x4: SB(32, 4)
        default: SB(64, 4)
    }
#undef SB
}

}  // namespace uhnsw
