// Device code of the U-HNSW query path on gfx950 (U-HNSW paper, Sec. 3.1
// and Algorithm 1), shared by the kernel translation units: the walk, fused
// and descent kernels are instantiated per (storage, index variant) in
// uhnsw_walk_part.hip, the verification and utility kernels in
// uhnsw_kernels.hip. One 64-lane wavefront serves one query; each wave keeps
// its state in its own slice of LDS, so waves of one workgroup never wait for
// each other.
//
//   walk   : graph choice, greedy descent over the upper layers, layer-0
//            best-first search with the sorted candidate list W in LDS, C out.
//   verify : batched L_p verification of C with the tau early stop.
//
// Base distances follow one fixed FP32 order: element j is accumulated by
// lane (j / V) % G of a G-lane group in ascending j (L2 by fused
// multiply-add), and the G lanes combine pairwise (lane l < o takes
// s_l + s_{l+o}, o = G/2 .. 1). Rows are zero-padded to G*V*NCH elements,
// which adds exact zeros only.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "uhnsw_internal.h"

namespace uhnsw {

// ------------------------------------------------------------ wave helpers
// Orders this wave's LDS accesses across lanes: LDS operations of one wave
// execute in program order, so a compiler-level fence is all that is needed.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool b) { return __ballot(b); }

__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ bool key_less(float ka, uint32_t ia, float kb, uint32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

// Pairwise combine inside a G-lane group; lane l < o receives s_l + s_{l+o}
// (o = G/2 .. 1), every lane of the group ends with the group's sum.
template <int G>
__device__ __forceinline__ float group_sum(float s) {
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) s = s + __shfl_xor(s, o, kWave);
    return s;
}

// The same combine, in the same order, where only lane 0 of each group needs
// the sum (the other lanes end with partial values): steps inside a 16-lane
// row read lane l + o with a DPP row shift, one VALU instruction each, and
// no LDS round trip; wider steps use a cross-lane permute.
template <int O>
__device__ __forceinline__ float shift_down(float s) {
    if constexpr (O >= 16)
        return __shfl_down(s, O, kWave);
    else  // row_shl:O (DPP control 0x100 + O): lane l reads lane l + O of its row
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(s), 0x100 + O, 0xF, 0xF, true));
}

template <int G>
__device__ __forceinline__ float group_sum_lane0(float s) {
    if constexpr (G > 1) {
        s = s + shift_down<G / 2>(s);
        return group_sum_lane0<G / 2>(s);
    }
    return s;
}

// Wave-wide minimum of (key, id); every lane gets the result.
__device__ __forceinline__ void wave_argmin(float &k, int32_t &id) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        float ko = __shfl_xor(k, o, kWave);
        int32_t io = __shfl_xor(id, o, kWave);
        if (key_less(ko, (uint32_t)io, k, (uint32_t)id)) {
            k = ko;
            id = io;
        }
    }
}

// ------------------------------------------------------- element loading
// Four consecutive elements per lane load. Loads land in `Raw` registers
// (packed 16-bit pairs for BF16 / FP16, so a row in flight costs half the
// VGPRs) and are widened exactly to FP32 only when used.
template <typename T>
struct Elem;
template <>
struct Elem<float> {
    using Raw = float4;
    __device__ static __forceinline__ Raw load(const float *p) { return *reinterpret_cast<const float4 *>(p); }
    __device__ static __forceinline__ Raw zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ static __forceinline__ void widen(const Raw &v, float (&x)[4]) {
        x[0] = v.x;
        x[1] = v.y;
        x[2] = v.z;
        x[3] = v.w;
    }
    __device__ static __forceinline__ void load4(const float *p, float (&x)[4]) { widen(load(p), x); }
};
struct bf16_t {
    uint16_t b;
};
struct f16_t {
    uint16_t b;
};
template <>
struct Elem<bf16_t> {
    using Raw = uint2;
    __device__ static __forceinline__ Raw load(const bf16_t *p) { return *reinterpret_cast<const uint2 *>(p); }
    __device__ static __forceinline__ Raw zero() { return make_uint2(0u, 0u); }
    __device__ static __forceinline__ void widen(const Raw &v, float (&x)[4]) {
        x[0] = __uint_as_float(v.x << 16);
        x[1] = __uint_as_float(v.x & 0xffff0000u);
        x[2] = __uint_as_float(v.y << 16);
        x[3] = __uint_as_float(v.y & 0xffff0000u);
    }
};
template <>
struct Elem<f16_t> {
    using Raw = uint2;
    __device__ static __forceinline__ Raw load(const f16_t *p) { return *reinterpret_cast<const uint2 *>(p); }
    __device__ static __forceinline__ Raw zero() { return make_uint2(0u, 0u); }
    __device__ static __forceinline__ void widen(const Raw &v, float (&x)[4]) {
        x[0] = __half2float(__ushort_as_half((unsigned short)(v.x & 0xffffu)));
        x[1] = __half2float(__ushort_as_half((unsigned short)(v.x >> 16)));
        x[2] = __half2float(__ushort_as_half((unsigned short)(v.y & 0xffffu)));
        x[3] = __half2float(__ushort_as_half((unsigned short)(v.y >> 16)));
    }
};

// ----------------------------------------------------------- base metric
// Base metrics of the walk: L1, squared L2, and L0.5 as sum sqrt|x - q| (the
// L0.5 distance is its square; the extended index of Sec. 4.5 walks G_0.5
// under it). Each lane sums its elements in ascending order, then the lane
// group combines pairwise.
// kMetL05F: the same key when every nonzero |x - q| is at least 2^-95 (the
// host and the query checks guarantee it), rooted by sqrt_rn_large.
// kMetL05T: the same key when every value is an integer in [0, 255] (so is
// |x - q|): the roots come from a 256-entry table of sqrtf(i) in LDS.
// kMetLp: sum |x - q|^pw for a fixed pw (a graph built for one p, the
// per-p HNSW of Sec. 4.3), each term exp2(pw log2|x - q|) on v_log_f32 /
// v_exp_f32 as in the verification.
constexpr int kMetL1 = 1, kMetL2 = 2, kMetL05 = 3, kMetL05F = 4, kMetL05T = 5, kMetLp = 6;
// how the graph-0 key of an extended-kernel query is taken: the L0.5 roots
// (see above), or kRootPow: the per-p variant's sum |x - q|^walk_p
constexpr int kRootSqrtf = 0, kRootShort = 1, kRootTable = 2, kRootPow = 3;
constexpr int kRootTableBytes = 256 * 4;
// descent pre-pass LDS per wave: 64 ids + 64 keys (+ the root table)
__host__ __device__ constexpr int descend_lds_wave_bytes(bool ext) { return 512 + (ext ? kRootTableBytes : 0); }

// Magnitude at or above which a nonzero base or query value keeps every
// nonzero difference with another such value (or with 0) at or above
// 2^-95: the difference is a multiple of the smaller operand's ulp.
constexpr float kL05FastMin = 0x1p-72f;

// Square root rounded to nearest for x = 0, +inf or x >= 2^-96. The
// hardware root r is within one ulp of the true root, so the rounded root is
// r - ulp, r or r + ulp; the signs of the residuals x - (r - ulp) r and
// x - (r + ulp) r, each exact in sign through one fused multiply-add (no
// underflow at these magnitudes), pick it.
__device__ __forceinline__ float sqrt_rn_large(float x) {
    const float r = __builtin_amdgcn_sqrtf(x);
    const float rm = __uint_as_float(__float_as_uint(r) - 1u);
    const float rp = __uint_as_float(__float_as_uint(r) + 1u);
    const float y = __builtin_fmaf(-rm, r, x) <= 0.0f ? rm : r;
    return __builtin_fmaf(-rp, r, x) > 0.0f ? rp : y;
}

// keys[r] = delta(row ids[r], q) for r < nrows. All lanes must call. The
// loads of up to RB row-steps are issued before any arithmetic so that a
// whole neighbour list is in flight at once.
template <int G, int NCH, typename T, int MET, int RBV>
__device__ __forceinline__ void rows_base_dist(const T *__restrict__ base, int64_t pitch,
                                               const int32_t *ids, int nrows, const float (&qv)[NCH][4],
                                               float *keys, const float *sqt = nullptr, float pw = 0.0f) {
    constexpr int V = 4;
    constexpr int RPW = kWave / G;
    constexpr int RB = (RBV * 4 / (NCH * V * (int)sizeof(T))) > 0 ? (RBV * 4 / (NCH * V * (int)sizeof(T))) : 1;
    using E = Elem<T>;
    const int lane = lane_id();
    const int grp = lane / G, gl = lane % G;
    for (int r0 = 0; r0 < nrows; r0 += RPW * RB) {
        // row-steps holding at least one row (a wave-uniform count): the
        // others are neither loaded nor summed. Lanes past the last row load
        // a copy of it (the same lines as its own group, so no extra
        // traffic) and their sums are dropped.
        const int left = nrows - r0;
        typename E::Raw raw[RB][NCH];
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            if (b == 0 || b * RPW < left) {
                const int row = min(r0 + b * RPW + grp, nrows - 1);
                const T *rp = base + (int64_t)ids[row] * pitch + gl * V;
#pragma unroll
                for (int c = 0; c < NCH; ++c) raw[b][c] = E::load(rp + c * G * V);
            }
        }
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            if (!(b == 0 || b * RPW < left)) break;
            float s = 0.0f;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                float x[V];
                E::widen(raw[b][c], x);
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const float dlt = x[e] - qv[c][e];
                    if (MET == kMetL1)
                        s = s + fabsf(dlt);
                    else if (MET == kMetL2)
                        s = __builtin_fmaf(dlt, dlt, s);
                    else if (MET == kMetL05F)
                        s = s + sqrt_rn_large(fabsf(dlt));
                    else if (MET == kMetL05T)
                        s = s + sqt[(int)fabsf(dlt)];
                    else if (MET == kMetLp)
                        s = s + __builtin_amdgcn_exp2f(pw * __builtin_amdgcn_logf(fabsf(dlt)));
                    else
                        s = s + sqrtf(fabsf(dlt));  // correctly rounded root
                }
            }
            s = group_sum_lane0<G>(s);
            const int row = r0 + b * RPW + grp;
            if (row < nrows && gl == 0) keys[row] = s;
        }
    }
}

// lo: the query walks graph 0 (G1, or G_0.5 / G_p when EXT) rather than
// graph 1 (G2, or G_1 / the L2 graph when EXT). root (EXT only): how the
// graph-0 key is taken, kRootTable reading sqt (LDS), kRootShort the short
// correctly rounded root, kRootPow the per-p variant's power pw (graph 1 is
// then walked under L2).
template <int G, int NCH, typename T, int RBV, bool EXT>
__device__ __forceinline__ void base_dists(bool lo, int root, const float *sqt, const T *base, int64_t pitch,
                                           const int32_t *ids, int nrows, const float (&qv)[NCH][4],
                                           float *keys, float pw) {
    if (EXT && root == kRootPow) {
        if (lo)
            rows_base_dist<G, NCH, T, kMetLp, RBV>(base, pitch, ids, nrows, qv, keys, nullptr, pw);
        else
            rows_base_dist<G, NCH, T, kMetL2, RBV>(base, pitch, ids, nrows, qv, keys);
    } else if (EXT && lo && root == kRootTable)
        rows_base_dist<G, NCH, T, kMetL05T, RBV>(base, pitch, ids, nrows, qv, keys, sqt);
    else if (EXT && lo && root == kRootShort)
        rows_base_dist<G, NCH, T, kMetL05F, RBV>(base, pitch, ids, nrows, qv, keys);
    else if (lo)
        rows_base_dist<G, NCH, T, EXT ? kMetL05 : kMetL1, RBV>(base, pitch, ids, nrows, qv, keys);
    else
        rows_base_dist<G, NCH, T, EXT ? kMetL1 : kMetL2, RBV>(base, pitch, ids, nrows, qv, keys);
}

// --------------------------------------------------- sorted-list insert
// L (keys Lk, ids Li; ids may carry kExpBit) holds nL entries ascending by
// (key, id). Insert the nU entries of (Uk, Ui) (any order, ids without the
// bit), drop those already present, keep the first cap entries. Scratch:
// Ulo, Urank, Slo, each nU ints. Returns the new size; *min_new receives the
// smallest position any new entry took (cap if none); *n_in the number of
// new entries now in L. With dedupe_u, an id listed twice in U is kept once
// (U holds at most kUCap entries then).
// WIDE selects the walk's form: a four-way search and a rank loop that issues
// its reads ahead, worth their extra registers on W's up to 1,024 entries;
// verification's short lists use plain halving.
template <bool WIDE>
__device__ int merge_into_sorted(float *Lk, uint32_t *Li, int nL, int cap, const float *Uk, const int32_t *Ui,
                                 int nU, int32_t *Ulo, int32_t *Urank, int32_t *Slo, bool dedupe_u, int *min_new,
                                 int *n_in) {
    const int lane = lane_id();
    // 1. insertion point of each candidate; -1 marks a duplicate
    // (lower bound by a four-way search: three pivots read together per step,
    // so the dependent LDS round trips are about half those of halving)
    for (int u = lane; u < nU; u += kWave) {
        const float uk = Uk[u];
        const uint32_t ui = (uint32_t)Ui[u];
        int lo = 0, hi = nL;
        while (WIDE && hi - lo >= 4) {
            const int q = (hi - lo) >> 2;
            const int m1 = lo + q, m2 = lo + 2 * q, m3 = lo + 3 * q;
            const float k1 = Lk[m1], k2 = Lk[m2], k3 = Lk[m3];
            const uint32_t i1 = Li[m1] & kIdMask, i2 = Li[m2] & kIdMask, i3 = Li[m3] & kIdMask;
            const bool c1 = key_less(k1, i1, uk, ui), c2 = key_less(k2, i2, uk, ui), c3 = key_less(k3, i3, uk, ui);
            if (c3) {
                lo = m3 + 1;
            } else if (c2) {
                lo = m2 + 1;
                hi = m3;
            } else if (c1) {
                lo = m1 + 1;
                hi = m2;
            } else {
                hi = m1;
            }
        }
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (key_less(Lk[mid], Li[mid] & kIdMask, uk, ui))
                lo = mid + 1;
            else
                hi = mid;
        }
        const bool dup = lo < nL && (Li[lo] & kIdMask) == ui;
        Ulo[u] = (dup || lo >= cap) ? -1 : lo;
    }
    wave_sync();
    if (dedupe_u) {  // keep the first copy of an id listed twice in U
        bool drop[(kUCap + kWave - 1) / kWave] = {};
        for (int u0 = 0, w = 0; u0 < nU && w < (kUCap + kWave - 1) / kWave; u0 += kWave, ++w) {
            const int u = u0 + lane;
            if (u < nU && Ulo[u] >= 0)
                for (int j = 0; j < u; ++j)
                    if (Ui[j] == Ui[u]) drop[w] = true;
        }
        wave_sync();
        for (int u0 = 0, w = 0; u0 < nU && w < (kUCap + kWave - 1) / kWave; u0 += kWave, ++w)
            if (u0 + lane < nU && drop[w]) Ulo[u0 + lane] = -1;
        wave_sync();
    }
    // 2. rank among the kept candidates
    int nkeep = 0;
    for (int u0 = 0; u0 < nU; u0 += kWave) {
        const int u = u0 + lane;
        int rank = -1;
        bool kept = false;
        if (u < nU && Ulo[u] >= 0) {
            kept = true;
            const float uk = Uk[u];
            const uint32_t ui = (uint32_t)Ui[u];
            rank = 0;
            if (WIDE) {
                // all three reads of an entry issued together, four entries
                // per step; no read waits on another entry's test
#pragma unroll 4
                for (int j = 0; j < nU; ++j) {
                    const int lj = Ulo[j];
                    const float kj = Uk[j];
                    const uint32_t ij = (uint32_t)Ui[j];
                    rank += ((lj >= 0) & ((kj < uk) | ((kj == uk) & (ij < ui)))) ? 1 : 0;
                }
            } else {
                for (int j = 0; j < nU; ++j)
                    if (Ulo[j] >= 0 && key_less(Uk[j], (uint32_t)Ui[j], uk, ui)) ++rank;
            }
        }
        if (u < nU) Urank[u] = rank;
        nkeep += popc64(ballot(kept));
    }
    wave_sync();
    *n_in = 0;
    *min_new = cap;
    if (nkeep == 0) return nL;
    for (int u = lane; u < nU; u += kWave)
        if (Urank[u] >= 0) Slo[Urank[u]] = Ulo[u];
    wave_sync();
    const int first = Slo[0];
    // 3. move the old entries at positions >= first to the right, top chunk first
    for (int cs = ((nL - 1) / kWave) * kWave; cs >= 0 && cs + kWave > first; cs -= kWave) {
        const int i = cs + lane;
        const bool act = i >= first && i < nL;
        float k = 0.0f;
        uint32_t id = 0;
        int ni = cap;
        if (act) {
            k = Lk[i];
            id = Li[i];
            int a = 0, b = nkeep;
            while (a < b) {
                const int m = (a + b) >> 1;
                if (Slo[m] <= i)
                    a = m + 1;
                else
                    b = m;
            }
            ni = i + a;
        }
        wave_sync();
        if (act && ni < cap) {
            Lk[ni] = k;
            Li[ni] = id;
        }
        wave_sync();
    }
    // 4. place the new entries
    int nin = 0;
    for (int u0 = 0; u0 < nU; u0 += kWave) {
        const int u = u0 + lane;
        bool in = false;
        if (u < nU && Urank[u] >= 0) {
            const int np = Ulo[u] + Urank[u];
            if (np < cap) {
                Lk[np] = Uk[u];
                Li[np] = (uint32_t)Ui[u];
                in = true;
            }
        }
        nin += popc64(ballot(in));
    }
    wave_sync();
    *n_in = nin;
    *min_new = first;
    const int nn = nL + nkeep;
    return nn < cap ? nn : cap;
}

// ------------------------------------------------- the walk's list merge
// (key, id) as one unsigned 64-bit value with the same order: keys are +0,
// positive or +inf (sums of nonnegative terms), so their bits order as
// unsigned integers; the expanded bit is not part of the id.
__device__ __forceinline__ uint64_t pack_key(float k, uint32_t id) {
    return ((uint64_t)__float_as_uint(k) << 32) | (id & kIdMask);
}
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

// New entries at most this many are placed one at a time by the whole wave.
constexpr int kFewNew = 4;

// Insert into the walk's list W (keys Lk, ids Li with the expanded bit, nL
// entries ascending by (key, id)) the new entries held in registers: entry
// (uk, ui) on each lane of the mask um, no expanded bit. Entries already in W
// are dropped, and with dedupe_u a second copy of an id in the mask; the
// first cap entries are kept. Returns the new size; *min_new receives the
// smallest position a new entry took (cap if none), *n_in the number of new
// entries now in W.
//
// Each new entry's insertion point: with at most kFewNew entries, the wave
// places one entry at a time: lanes 0..31 hold every B-th entry of W (the
// last of each block of B, B = 8 .. 64 so that 32 blocks cover W), one
// ballot of "pivot below the entry" gives its block, one read of that block
// (one entry per lane) and a ballot give its position and whether W holds it
// -- two LDS round trips in all. More entries search W lane by lane. Ranks
// among the kept entries and the shift of W's tail are counted from
// registers (lane reads), and the tail moves in groups of up to 256 entries:
// read together, then written.
// on_first(first, id): called once the kept entries are ranked, with the
// first position a new entry takes and that entry's id (the walk fetches
// its neighbours early when it will be the next pick).
template <bool WIDE, typename OnFirst>
__device__ int merge_walk(float *Lk, uint32_t *Li, int nL, int cap, float uk, uint32_t ui, uint64_t um,
                          bool dedupe_u, int *min_new, int *n_in, OnFirst on_first) {
    const int lane = lane_id();
    const uint64_t u = ((um >> lane) & 1ull) ? pack_key(uk, ui) : ~0ull;
    if (dedupe_u) {  // keep the lowest lane of an id listed twice
        bool drop = false;
        for (uint64_t m = um; m; m &= m - 1) {
            const int j = __builtin_ctzll(m);
            drop = drop || (((um >> lane) & 1ull) && lane > j && readlane64(u, j) == u);
        }
        um &= ~ballot(drop);
    }
    const bool mine = (um >> lane) & 1ull;
    *n_in = 0;
    *min_new = cap;
    const int nU = popc64(um);
    if (nU == 0) return nL;
    int lo = 0;
    bool dup = false;
    if (nU <= kFewNew) {
        int B = 8;
        while (B * 32 < nL) B <<= 1;
        const int ppos = (lane + 1) * B - 1;
        const uint64_t piv = (lane < 32 && ppos < nL) ? pack_key(Lk[ppos], Li[ppos]) : ~0ull;
        uint64_t m = um;
#pragma unroll
        for (int jj = 0; jj < kFewNew; ++jj) {
            if (m == 0) break;
            const int j = __builtin_ctzll(m);
            m &= m - 1;
            const uint64_t uj = readlane64(u, j);
            const int blk = popc64(ballot(piv < uj));  // pivots ascend: the ones below form a prefix
            const int e = blk * B + lane;
            const uint64_t w = (lane < B && e < nL) ? pack_key(Lk[e], Li[e]) : ~0ull;
            const int loj = blk * B + popc64(ballot(w < uj));
            const bool dj = ballot(w == uj) != 0ull;
            if (lane == j) {
                lo = loj;
                dup = dj;
            }
        }
    } else if (mine) {
        int a = 0, b = nL;
        while (WIDE && b - a >= 4) {  // three pivots read together per step
            const int q = (b - a) >> 2;
            const int m1 = a + q, m2 = a + 2 * q, m3 = a + 3 * q;
            const uint64_t p1 = pack_key(Lk[m1], Li[m1]), p2 = pack_key(Lk[m2], Li[m2]), p3 = pack_key(Lk[m3], Li[m3]);
            if (p3 < u) {
                a = m3 + 1;
            } else if (p2 < u) {
                a = m2 + 1;
                b = m3;
            } else if (p1 < u) {
                a = m1 + 1;
                b = m2;
            } else {
                b = m1;
            }
        }
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (pack_key(Lk[mid], Li[mid]) < u)
                a = mid + 1;
            else
                b = mid;
        }
        lo = a;
        dup = a < nL && pack_key(Lk[a], Li[a]) == u;
    }
    const bool keep = mine && !dup && lo < cap;
    const uint64_t km = ballot(keep);
    if (km == 0) return nL;
    const int nkeep = popc64(km);
    // rank among the kept entries; the first position any of them takes
    int rank = 0, first = cap;
    for (uint64_t m = km; m; m &= m - 1) {
        const int j = __builtin_ctzll(m);
        rank += readlane64(u, j) < u ? 1 : 0;
        first = min(first, __builtin_amdgcn_readlane(lo, j));
    }
    on_first(first, (uint32_t)__builtin_amdgcn_readlane((int)ui, __builtin_ctzll(ballot(keep && rank == 0))));
    // move W's entries at positions >= first right by the number of kept
    // entries placed at or before them, the top group first
    for (int top = nL; top > first; top -= 4 * kWave) {
        const int g0 = max(first, top - 4 * kWave);
        float k[4];
        uint32_t id[4];
        int sh[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = g0 + c * kWave + lane;
            sh[c] = 0;
            if (i < top) {
                k[c] = Lk[i];
                id[c] = Li[i];
            }
        }
        for (uint64_t m = km; m; m &= m - 1) {
            const int lj = __builtin_amdgcn_readlane(lo, __builtin_ctzll(m));
#pragma unroll
            for (int c = 0; c < 4; ++c) sh[c] += lj <= g0 + c * kWave + lane ? 1 : 0;
        }
        wave_sync();
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = g0 + c * kWave + lane;
            if (i < top && i + sh[c] < cap) {
                Lk[i + sh[c]] = k[c];
                Li[i + sh[c]] = id[c];
            }
        }
        wave_sync();
    }
    // place the kept entries
    const int np = lo + rank;
    const bool in = keep && np < cap;
    if (in) {
        Lk[np] = uk;
        Li[np] = ui;
    }
    wave_sync();
    *n_in = popc64(ballot(in));
    *min_new = first;
    const int nn = nL + nkeep;
    return nn < cap ? nn : cap;
}

// Visited cache: a table in LDS that never reports a node as visited unless
// it was (it may forget; a forgotten node is gathered again and dropped
// against W, or is worse than W's last entry). Two slot formats:
//  * 16-bit tags when ids fit (vis_tags_fit): h = id * odd mod 2^kbits is a
//    bijection on kbits-bit values; the tags form sets of kVisWays (one LDS
//    word of 2 * kVisWays bytes, read in one access), the top bits of h pick
//    the set and the remaining bits + 1 are the tag (0 empty) -- set and tag
//    together identify the id, so a tag match is exact. An insert shifts the
//    set's tags up by one (the oldest falls out) and puts the new tag at the
//    bottom; two inserts into one set in the same step both start from the
//    set the probe read, so one of them is lost (a forgotten node, never a
//    false one);
//  * 32-bit slots holding the id (-1 empty), direct-mapped by a
//    multiplicative hash (ids too wide for the tags).
// Sets of 8 (one 16-byte read per probe): on the 1M x 128 workload at ef 256
// the walk gathers 4,395 rows per query where a direct-mapped table of the
// same 8 KiB gathers 4,940 and an exact visited set 4,209; the walk, at the
// random-gather ceiling of HBM, runs 8 % faster (4-way: 4,496 rows, 7 %).
template <int W> struct VisWord;
template <> struct VisWord<1> { using T = uint16_t; };
template <> struct VisWord<2> { using T = uint32_t; };
template <> struct VisWord<4> { using T = uint2; };
template <> struct VisWord<8> { using T = uint4; };

__device__ __forceinline__ uint32_t vis_zero16(uint32_t x) { return (x - 0x00010001u) & ~x & 0x80008000u; }
__device__ __forceinline__ bool vis_has(uint16_t w, uint32_t tt) { return (uint32_t)w == (tt & 0xffffu); }
__device__ __forceinline__ bool vis_has(uint32_t w, uint32_t tt) { return vis_zero16(w ^ tt) != 0u; }
__device__ __forceinline__ bool vis_has(uint2 w, uint32_t tt) { return (vis_zero16(w.x ^ tt) | vis_zero16(w.y ^ tt)) != 0u; }
__device__ __forceinline__ bool vis_has(uint4 w, uint32_t tt) {
    return (vis_zero16(w.x ^ tt) | vis_zero16(w.y ^ tt) | vis_zero16(w.z ^ tt) | vis_zero16(w.w ^ tt)) != 0u;
}
__device__ __forceinline__ uint16_t vis_push(uint16_t, uint32_t t) { return (uint16_t)t; }
__device__ __forceinline__ uint32_t vis_push(uint32_t w, uint32_t t) { return (w << 16) | t; }
__device__ __forceinline__ uint2 vis_push(uint2 w, uint32_t t) { return make_uint2((w.x << 16) | t, (w.y << 16) | (w.x >> 16)); }
__device__ __forceinline__ uint4 vis_push(uint4 w, uint32_t t) {
    return make_uint4((w.x << 16) | t, (w.y << 16) | (w.x >> 16), (w.z << 16) | (w.y >> 16), (w.w << 16) | (w.z >> 16));
}

struct VisCache {
    void *base;
    int bits, kbits;

    __device__ __forceinline__ void clear(int lane) const {
        const int words = kbits ? (1 << bits) / 2 : (1 << bits);
        const int32_t fill = kbits ? 0 : -1;
        int32_t *w = reinterpret_cast<int32_t *>(base);
        for (int i = lane; i < words; i += kWave) w[i] = fill;
    }
    // slot: the set (tag format) or the slot (id format)
    __device__ __forceinline__ void locate(int32_t id, uint32_t &slot, uint32_t &tag) const {
        if (kbits) {
            const int sbits = bits - kVisWayBits;
            const uint32_t h = ((uint32_t)id * 0x9E3779B1u) & ((kbits == 32 ? 0u : (1u << kbits)) - 1u);
            slot = h >> (kbits - sbits);
            tag = (h & ((1u << (kbits - sbits)) - 1u)) + 1u;
        } else {
            slot = ((uint32_t)id * 2654435761u) >> (32 - bits);
            tag = (uint32_t)id;
        }
    }
    // probe and, if absent, insert: returns whether the node was absent
    __device__ __forceinline__ bool test_and_mark(uint32_t slot, uint32_t tag) const {
        if (kbits) {
            using T = typename VisWord<kVisWays>::T;
            T *sets = reinterpret_cast<T *>(base);
            const T w = sets[slot];
            if (vis_has(w, tag * 0x00010001u)) return false;
            sets[slot] = vis_push(w, tag);
            return true;
        }
        uint32_t *slots = reinterpret_cast<uint32_t *>(base);
        if (slots[slot] == tag) return false;
        slots[slot] = tag;
        return true;
    }
    // the first node of a walk, into an empty cache
    __device__ __forceinline__ void mark_first(int32_t id) const {
        uint32_t s, t;
        locate(id, s, t);
        test_and_mark(s, t);
    }
};

// ------------------------------------------------------------------- walk
// Per wave: W (keys, then ids), the visited cache, the new rows' ids and keys
// (kUCap each), and for the extended index the L0.5 root table.
struct WalkLds {
    float *Wk;
    uint32_t *Wi;
    VisCache vis;
    int32_t *Uid;
    float *Uk;
    float *sqt;
};

__host__ __device__ inline int vis_bytes_impl(int vis_bits, int vis_kbits) {
    return (1 << vis_bits) * (vis_kbits ? 2 : 4);
}

// ext: the extended index's walk also holds the L0.5 root table
__host__ __device__ inline int walk_lds_bytes_impl(int ef_cap, int vis_bits, int vis_kbits, bool ext) {
    return ef_cap * 8 + vis_bytes_impl(vis_bits, vis_kbits) + kUCap * 4 * 2 + (ext ? kRootTableBytes : 0);
}

__device__ inline WalkLds walk_lds(char *p, int ef_cap, int vis_bits, int vis_kbits) {
    WalkLds L;
    L.Wk = reinterpret_cast<float *>(p);
    L.Wi = reinterpret_cast<uint32_t *>(L.Wk + ef_cap);
    L.vis.base = L.Wi + ef_cap;
    L.vis.bits = vis_bits;
    L.vis.kbits = vis_kbits;
    L.Uid = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(L.vis.base) + vis_bytes_impl(vis_bits, vis_kbits));
    L.Uk = reinterpret_cast<float *>(L.Uid + kUCap);
    L.sqt = L.Uk + kUCap;  // extended walk only
    return L;
}

// p outside the index's range ([0.5, 2]; [0.2, 1] for the extended pair)
// or NaN, K or ef outside their bounds.
template <bool EXT>
__device__ __forceinline__ bool query_bad(const SearchArgs &A, float p, int K, int ef) {
    const bool p_ok = p >= A.p_lo && p <= A.p_hi;
    return !p_ok || K < 1 || K > A.k_max || K > UHNSW_KMAX || ef < K || ef > A.ef_max || ef > A.ef_cap;
}

// An integer in [0, 255]: with every base value such too (checked on the
// host), each |x - q| indexes the root table exactly.
__device__ __forceinline__ bool is_byte_value(float v) { return v >= 0.0f && v <= 255.0f && v == rintf(v); }

// The L0.5 root form of one query (wave-uniform inputs): the table when the
// index and the query hold byte values (the table is filled here: 256
// correctly rounded roots), else the short form when no difference can fall
// below 2^-95, else sqrtf.
__device__ __forceinline__ int l05_root_mode(const SearchArgs &A, bool no_tiny, bool bytes, float *sqt) {
    if (A.walk_p > 0.0f) return kRootPow;  // the per-p variant
    if (A.l05_table && bytes) {
        for (int i = lane_id(); i < 256; i += kWave) sqt[i] = sqrtf((float)i);
        wave_sync();
        return kRootTable;
    }
    return A.l05_fast && no_tiny ? kRootShort : kRootSqrtf;
}

// Greedy descent over layers max_level .. 1 of graph Gr from its entry
// point, always to the smallest (key, id) neighbour; returns the layer-0
// entry node and its key, and adds the base distances computed to *n_b.
// Uid / Uk: 64-entry LDS scratch of the wave.
template <int G, int NCH, typename T, int RBV, bool EXT>
__device__ int32_t descend(const DevGraph &Gr, bool lo, int root, const float *sqt, const T *base, int64_t pitch,
                           const float (&qv)[NCH][4], int32_t *Uid, float *Uk, float *kout, int *n_b, float pw) {
    const int lane = lane_id();
    int32_t cur = Gr.entry;
    if (lane == 0) Uid[0] = cur;
    wave_sync();
    base_dists<G, NCH, T, RBV, EXT>(lo, root, sqt, base, pitch, Uid, 1, qv, Uk, pw);
    wave_sync();
    float kcur = Uk[0];
    *n_b += 1;
    for (int l = Gr.max_level; l >= 1; --l) {
        for (;;) {
            wave_sync();
            const int64_t row = (int64_t)Gr.up_off[cur] + (l - 1);
            const int32_t nb = lane < Gr.M ? Gr.up_adj[row * Gr.M + lane] : -1;
            const int cnt = popc64(ballot(nb >= 0));
            if (nb >= 0) Uid[lane] = nb;  // valid ids come first in each row
            wave_sync();
            base_dists<G, NCH, T, RBV, EXT>(lo, root, sqt, base, pitch, Uid, cnt, qv, Uk, pw);
            wave_sync();
            *n_b += cnt;
            float kb = lane < cnt ? Uk[lane] : INFINITY;
            int32_t ib = lane < cnt ? Uid[lane] : 0x7fffffff;
            wave_argmin(kb, ib);
            if (cnt > 0 && key_less(kb, (uint32_t)ib, kcur, (uint32_t)cur)) {
                cur = ib;
                kcur = kb;
            } else {
                break;
            }
        }
    }
    *kout = kcur;
    return cur;
}

// The query slice of this lane (elements c*G*4 + (lane % G)*4 + e), zero
// beyond d.
template <int G, int NCH>
__device__ __forceinline__ void load_query(const float *q, int d, float (&qv)[NCH][4]) {
    const int gl = lane_id() % G;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = c * G * 4 + gl * 4 + e;
            qv[c][e] = j < d ? q[j] : 0.0f;
        }
}

template <int G, int NCH, typename T, int RBV, bool WIDE, bool EXT>
__device__ __forceinline__ int walk_one(const SearchArgs &A, int64_t qi, char *lds) {
    const int lane = lane_id();
    const uint32_t t_begin = (uint32_t)wall_clock64();
    const WalkLds L = walk_lds(lds, A.ef_cap, A.vis_bits, A.vis_kbits);
    const float p = A.p[qi];
    const int K = A.k[qi];
    const int ef = A.ef[qi];
    uhnsw_stats *st = A.stats + qi;
    int32_t *cid = A.cand_ids ? A.cand_ids + qi * A.c_stride : nullptr;
    float *ckey = A.cand_keys ? A.cand_keys + qi * A.c_stride : nullptr;
    bool finite = true, tiny = false, byte = true;
    for (int j = lane; j < A.d; j += kWave) {
        const float v = A.queries[qi * A.d + j];
        finite = finite && isfinite(v);
        if (EXT) {
            tiny = tiny || (v != 0.0f && fabsf(v) < kL05FastMin);
            byte = byte && is_byte_value(v);
        }
    }
    const bool bad = query_bad<EXT>(A, p, K, ef) || ballot(!finite) != 0;
    const int root = EXT ? l05_root_mode(A, ballot(tiny) == 0, ballot(!byte) == 0, L.sqt) : kRootSqrtf;
    if (bad) {
        if (cid)
            for (int i = lane; i < A.c_stride; i += kWave) {
                cid[i] = -1;
                ckey[i] = INFINITY;
            }
        if (lane == 0) {
            if (A.ncand) A.ncand[qi] = -1;
            st->graph = 0;
            st->n_b = st->n_exp = st->n_p = st->batches = st->nc = st->n_up = st->n_cut = 0;
            st->flags = UHNSW_QBAD;
            st->entry0 = -1;
            st->t_begin = st->t_end = t_begin;
        }
        return -1;
    }
    const int gsel = (p <= A.cutoff) ? 0 : 1;
    const DevGraph &Gr = A.g[gsel];
    const bool lo = gsel == 0;
    const int tp = A.t_param > 0 ? A.t_param : 6 * K;
    int t = ef < tp ? ef : tp;
    if (t < K) t = K;
    const T *base = reinterpret_cast<const T *>(A.walk_base);
    const int64_t pitch = A.pitch;

    float qv[NCH][4];
    load_query<G, NCH>(A.queries + qi * A.d, A.d, qv);
    L.vis.clear(lane);

    // ---- descent over the upper layers, unless a pre-pass already did it
    int32_t cur;
    float kcur;
    int n_b = 0;
    if (A.entry) {
        cur = A.entry[qi];
        kcur = A.ekey[qi];
        n_b = A.dnb[qi];
    } else {
        cur = descend<G, NCH, T, RBV, EXT>(Gr, lo, root, L.sqt, base, pitch, qv, L.Uid, L.Uk, &kcur, &n_b,
                                           A.walk_p);
    }
    const int32_t entry0 = cur;
    const int n_up = n_b;  // the descent's base distances

    // ---- layer 0: best-first expansion of the sorted list W
    wave_sync();
    if (lane == 0) {
        L.Wk[0] = kcur;
        L.Wi[0] = (uint32_t)cur;
        L.vis.mark_first(cur);
    }
    wave_sync();
    int nW = 1, lb = 0, n_exp = 0, flags = 0;
    int32_t spec_node = -1, spec_nb = -1;  // prefetched adjacency row (beam 1)
    const int M0 = Gr.M0;
    const int beam = A.beam;
    for (;;) {
        // the first `beam` (1 or 2) unexpanded entries, scanning from lb;
        // all values here are wave-uniform (LDS broadcast reads). With beam 1
        // the second unexpanded entry is found too: its adjacency row is
        // fetched early, and used if it turns out to be the next pick.
        int npick = 0, pos0 = -1, pos1 = -1, nseen = 0;
        uint32_t node0 = 0, node1 = 0;
        const int want = beam == 1 ? 2 : beam;
        for (int b0 = lb; b0 < nW && nseen < want; b0 += kWave) {
            const int i = b0 + lane;
            const uint32_t wi = i < nW ? L.Wi[i] : kExpBit;
            uint64_t m = ballot(!(wi & kExpBit));
            while (m && nseen < want) {
                const int l = __builtin_ctzll(m);
                m &= m - 1;
                // the entry is in lane l's register: no second LDS read
                const uint32_t node = (uint32_t)__builtin_amdgcn_readlane((int)wi, l);
                if (nseen == 0) {
                    pos0 = b0 + l;
                    node0 = node;
                } else {
                    pos1 = b0 + l;
                    node1 = node;
                }
                ++nseen;
            }
        }
        npick = beam == 1 ? (nseen > 0 ? 1 : 0) : nseen;
        if (npick == 0) break;
        if (n_exp >= A.n) {  // a valid walk expands each node at most once
            flags |= UHNSW_QCAP;
            break;
        }
        lb = pos0;
        wave_sync();
        if (lane == 0) {
            L.Wi[pos0] = node0 | kExpBit;
            if (npick > 1) L.Wi[pos1] = node1 | kExpBit;
        }
        n_exp += npick;
        // neighbours: lane = slot `lane % M0` of picked node `lane / M0`
        const int which = lane / M0, slot = lane % M0;
        int32_t nb = -1;
        if (beam == 1) {
            if ((int32_t)node0 == spec_node)
                nb = spec_nb;
            else if (which == 0)
                nb = Gr.adj0[(int64_t)node0 * M0 + slot];
            spec_node = nseen > 1 ? (int32_t)node1 : -1;
            if (nseen > 1 && which == 0) spec_nb = Gr.adj0[(int64_t)node1 * M0 + slot];
        } else if (which < npick) {
            nb = Gr.adj0[(int64_t)(which == 0 ? node0 : node1) * M0 + slot];
        }
        // probe, then mark what was not there: one LDS read and one write per
        // lane, each issued for all lanes at once, so every probe sees the
        // cache as it was before this step's marks
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
        base_dists<G, NCH, T, RBV, EXT>(lo, root, L.sqt, base, pitch, L.Uid, nnew, qv, L.Uk, A.walk_p);
        wave_sync();
        n_b += nnew;
        // the new entries, entry r on lane r
        const float nk = lane < nnew ? L.Uk[lane] : 0.0f;
        const uint32_t nid = lane < nnew ? (uint32_t)L.Uid[lane] : 0u;
        uint64_t um = nnew >= kWave ? ~0ull : ((1ull << nnew) - 1ull);
        // With W full, a new entry not below W's last one cannot enter. Late
        // in the walk most expansions end here with nothing to merge.
        if (nW == ef) {
            const uint64_t wl = pack_key(L.Wk[nW - 1], L.Wi[nW - 1]);
            um = ballot(lane < nnew && pack_key(nk, nid) < wl);
            if (um == 0) continue;
        }
        wave_sync();
        int min_new, n_in;
        // beam 1: the next pick is the smallest new entry if it lands at or
        // before the second unexpanded entry, else that entry (whose
        // neighbours are already in flight); fetch the new one's now
        const int pos_next = nseen > 1 ? pos1 : ef;
        nW = merge_walk<WIDE>(L.Wk, L.Wi, nW, ef, nk, nid, um, npick > 1, &min_new, &n_in,
                              [&](int first, uint32_t id0) {
                                  if (beam == 1 && first <= pos_next) {
                                      spec_node = (int32_t)id0;
                                      if (which == 0) spec_nb = Gr.adj0[(int64_t)id0 * M0 + slot];
                                  }
                              });
        if (min_new < lb) lb = min_new;
    }

    // ---- C = first t of W
    const int nc = nW < t ? nW : t;
    if (cid)
        for (int i = lane; i < A.c_stride; i += kWave) {
            cid[i] = i < nc ? (int32_t)(L.Wi[i] & kIdMask) : -1;
            ckey[i] = i < nc ? L.Wk[i] : INFINITY;
        }
    if (lane == 0) {
        if (A.ncand) A.ncand[qi] = nc;
        st->graph = gsel + 1;
        st->n_b = n_b;
        st->n_up = n_up;
        st->n_exp = n_exp;
        st->nc = nc;
        st->flags = flags;
        st->entry0 = entry0;
        st->t_begin = t_begin;
    }
    return nc;
}

// Next query index for this wave from the work counter. Every lane issues
// the atomic (lane 0 adds 1, the others add 0) so that no lane-dependent
// branch precedes the broadcast; the broadcast takes lane 0's old value.
__device__ __forceinline__ int fetch_query(int32_t *counter) {
    const int v = atomicAdd(counter, lane_id() == 0 ? 1 : 0);
    return __builtin_amdgcn_readfirstlane(__shfl(v, 0, kWave));
}

// Occupancy target (waves per SIMD) and VGPRs given to row data in flight.
// FP32 rows: 4 waves with a whole 32-row neighbour list in flight (64 VGPRs);
// 16-bit rows: 32 VGPRs (a whole list as well) and 5 waves for rows of up to
// 256 dimensions, 4 for longer rows. Measured on the 1M x 128 workload, a
// fifth FP32 wave or a sixth 16-bit wave costs more in spills than it gains.
template <typename T, int G>
constexpr int walk_waves_per_eu() { return sizeof(T) == 4 ? 4 : (G <= 16 ? 5 : 4); }
template <typename T>
constexpr int walk_rb_vgprs() { return sizeof(T) == 4 ? 64 : 32; }
template <int G, int NCH, typename T, bool EXT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(walk_waves_per_eu<T, G>(), 8))) walk_kernel(SearchArgs A) {
    extern __shared__ __attribute__((aligned(16))) char lds_all[];
    const int wave = threadIdx.x / kWave;
    char *lds = lds_all + (size_t)wave * A.lds_wave_bytes;
    if (A.counter == nullptr) {
        const int64_t k = (int64_t)blockIdx.x * A.waves_per_block + wave;
        if (k < A.nq) walk_one<G, NCH, T, walk_rb_vgprs<T>(), true, EXT>(A, A.order ? A.order[k] : k, lds);
        return;
    }
    // persistent: waves take queries from the counter until it passes nq
    int k = fetch_query(A.counter);
    while ((int64_t)k < A.nq) {
        const int64_t qi = A.order ? A.order[k] : k;
        walk_one<G, NCH, T, walk_rb_vgprs<T>(), true, EXT>(A, qi, lds);
        k = fetch_query(A.counter);
    }
}

// ----------------------------------------------------------------- verify
// L_p term |dlt|^p by class: 1 -> p = 1, 2 -> p = 2, 3 -> p = 0.5,
// 4 -> p = 1.5 (square roots, the paper's second cost class, Sec. 2.1),
// 0 -> any other p as exp2(p * log2|dlt|) on v_log_f32 / v_exp_f32.
template <int PC>
__device__ __forceinline__ float lp_acc(float s, float dlt, float p) {
    const float a = fabsf(dlt);
    if (PC == 1) return s + a;
    if (PC == 2) return __builtin_fmaf(dlt, dlt, s);
    if (PC == 3) return s + __builtin_amdgcn_sqrtf(a);
    if (PC == 4) return __builtin_fmaf(a, __builtin_amdgcn_sqrtf(a), s);
    return s + __builtin_amdgcn_exp2f(p * __builtin_amdgcn_logf(a));
}

// S[r] = sum |x - q|^p for the FP32 rows ids[r]. Every term is nonnegative
// and FP32 addition is monotone, so a partial sum (each lane's first chunks,
// combined over the group in the same pairwise order) never exceeds the full
// sum S; a row whose partial sum is already above thr (the K-th smallest S of
// R) cannot enter the top K. SPLIT (rows spread over 32 or 64 lanes, d > 256,
// four chunks per lane, abort on): the first half of each row is loaded and
// summed, and the second half is fetched only for rows whose partial sum is
// still at most thr; a row stopped there, or whose full S exceeds thr, is
// reported as +inf. Otherwise rows are loaded whole in one step and summed in
// full (rows of up to 256 dimensions: their few bytes are in flight together).
template <int G, int NCH, int PC, bool SPLIT>
__device__ __forceinline__ int rows_lp_impl(const float *__restrict__ base, int64_t pitch, const int32_t *ids,
                                             int nrows, const float (&qv)[NCH][4], float p, float thr, float *S) {
    constexpr int V = 4;
    constexpr int RPW = kWave / G;
    // verification batches are small (kappa rows): two row-steps in flight
    constexpr int RB = (32 / (NCH * V)) > 0 ? (32 / (NCH * V)) : 1;
    constexpr int H = SPLIT ? NCH / 2 : NCH;  // chunks loaded before the abort test
    const int lane = lane_id();
    const int grp = lane / G, gl = lane % G;
    int cut = 0;  // rows whose second half was not read
    for (int r0 = 0; r0 < nrows; r0 += RPW * RB) {
        float x[RB][NCH][V];
        const float *rp[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const int row = r0 + b * RPW + grp;
            rp[b] = row < nrows ? base + (int64_t)ids[row] * pitch + gl * V : nullptr;
#pragma unroll
            for (int c = 0; c < H; ++c) {
                if (rp[b])
                    Elem<float>::load4(rp[b] + c * G * V, x[b][c]);
                else
#pragma unroll
                    for (int e = 0; e < V; ++e) x[b][c][e] = qv[c][e];
            }
        }
        float s[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            s[b] = 0.0f;
#pragma unroll
            for (int c = 0; c < H; ++c)
#pragma unroll
                for (int e = 0; e < V; ++e) s[b] = lp_acc<PC>(s[b], x[b][c][e] - qv[c][e], p);
        }
        bool live[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) live[b] = true;
        if (SPLIT) {
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                // the group's partial sum, the same value on every lane of it
                live[b] = rp[b] != nullptr && !(group_sum<G>(s[b]) > thr);
                cut += popc64(ballot(gl == 0 && rp[b] != nullptr && !live[b]));
#pragma unroll
                for (int c = H; c < NCH; ++c) {
                    if (live[b])
                        Elem<float>::load4(rp[b] + c * G * V, x[b][c]);
                    else
#pragma unroll
                        for (int e = 0; e < V; ++e) x[b][c][e] = qv[c][e];
                }
            }
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int c = H; c < NCH; ++c)
#pragma unroll
                    for (int e = 0; e < V; ++e) s[b] = lp_acc<PC>(s[b], x[b][c][e] - qv[c][e], p);
        }
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const float t = group_sum_lane0<G>(s[b]);
            const int row = r0 + b * RPW + grp;
            if (row < nrows && gl == 0) S[row] = (SPLIT && (!live[b] || t > thr)) ? INFINITY : t;
        }
    }
    return cut;
}

// Returns the number of rows whose second half the abort left unread.
template <int G, int NCH, int PC>
__device__ __forceinline__ int rows_lp(const float *__restrict__ base, int64_t pitch, const int32_t *ids,
                                       int nrows, const float (&qv)[NCH][4], float p, float thr, bool abort,
                                       float *S) {
    if constexpr (G >= 32 && NCH >= 2) {
        if (abort) return rows_lp_impl<G, NCH, PC, true>(base, pitch, ids, nrows, qv, p, thr, S);
    }
    return rows_lp_impl<G, NCH, PC, false>(base, pitch, ids, nrows, qv, p, thr, S);
}

template <int G, int NCH>
__device__ __forceinline__ int lp_dists(int pc, const float *base, int64_t pitch, const int32_t *ids, int nrows,
                                        const float (&qv)[NCH][4], float p, float thr, bool abort, float *S) {
    switch (pc) {
        case 1: return rows_lp<G, NCH, 1>(base, pitch, ids, nrows, qv, p, thr, abort, S);
        case 2: return rows_lp<G, NCH, 2>(base, pitch, ids, nrows, qv, p, thr, abort, S);
        case 3: return rows_lp<G, NCH, 3>(base, pitch, ids, nrows, qv, p, thr, abort, S);
        case 4: return rows_lp<G, NCH, 4>(base, pitch, ids, nrows, qv, p, thr, abort, S);
        default: return rows_lp<G, NCH, 0>(base, pitch, ids, nrows, qv, p, thr, abort, S);
    }
}

// d_p = S^(1/p). For a general p the power is split so that the FP32 exp2
// sees a small argument: log2 S = e + log2 m with m in [1, 2) and e exact,
// e / p = n + r / p with n an integer and r = e - n p (one fused multiply-
// add), so S^(1/p) = 2^n * 2^((r + log2 m) / p) with |(r + log2 m) / p| <=
// 1/2 + 1/p. Taking exp2(log2(S) / p) directly loses accuracy in proportion
// to |log2 S| / p (1.1e-5 at S near 2^-11 and p = 0.2).
__device__ __forceinline__ float lp_root(float S, float p, int pc) {
    if (pc == 1) return S;
    if (pc == 2) return sqrtf(S);
    if (pc == 3) return S * S;
    if (!(S > 0.0f) || !isfinite(S)) return S;
    int e;
    const float m = 2.0f * frexpf(S, &e);  // S = m 2^(e-1), m in [1, 2)
    const float ef = (float)(e - 1);
    const float n = rintf(ef / p);
    const float r = __builtin_fmaf(-n, p, ef);
    return ldexpf(exp2f((r + log2f(m)) / p), (int)n);
}

struct VerifyLds {
    float *Rk;
    uint32_t *Ri;
    float *Bk;
    int32_t *Bi;
    int32_t *Ulo, *Urank, *Slo;
};

__host__ __device__ inline int verify_lds_bytes_impl(int kv_cap) { return kv_cap * 8 + kv_cap * 8 + kv_cap * 12; }

__device__ inline VerifyLds verify_lds(char *p, int kv_cap) {
    VerifyLds L;
    L.Rk = reinterpret_cast<float *>(p);
    L.Ri = reinterpret_cast<uint32_t *>(L.Rk + kv_cap);
    L.Bk = reinterpret_cast<float *>(L.Ri + kv_cap);
    L.Bi = reinterpret_cast<int32_t *>(L.Bk + kv_cap);
    L.Ulo = L.Bi + kv_cap;
    L.Urank = L.Ulo + kv_cap;
    L.Slo = L.Urank + kv_cap;
    return L;
}

// Verification of one query. C comes from global memory (Cg) or, in the
// fused kernel, straight from the walk's list in LDS (Cl, expanded bit set).
template <int G, int NCH>
__device__ __forceinline__ void verify_one(const SearchArgs &A, int64_t qi, char *lds, int nc, const int32_t *Cg,
                           const uint32_t *Cl) {
    const int lane = lane_id();
    const float p = A.p[qi];
    const int K = A.k[qi];
    const int ef = A.ef[qi];
    int64_t *oid = A.ids + qi * A.k_stride;
    float *odist = A.dists + qi * A.k_stride;
    uhnsw_stats *st = A.stats + qi;
    if (nc < 0) {  // rejected by the walk
        for (int r = lane; r < A.k_stride; r += kWave) {
            oid[r] = -1;
            odist[r] = INFINITY;
        }
        return;
    }
    (void)ef;
    const int kappa = A.kappa_param > 0 ? A.kappa_param : (K > 2 ? K : 2);
    const VerifyLds L = verify_lds(lds, A.kv_cap);
    const int pc = p == 1.0f ? 1 : p == 2.0f ? 2 : p == 0.5f ? 3 : p == 1.5f ? 4 : 0;
    const int m = A.mtab[K];
    float qv[NCH][4];
    {
        const int gl = lane % G;
        const float *q = A.queries + qi * A.d;
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = c * G * 4 + gl * 4 + e;
                qv[c][e] = j < A.d ? q[j] : 0.0f;
            }
    }
    // R = first K of C
    const int nR = nc < K ? nc : K;
    for (int i = lane; i < nR; i += kWave) L.Bi[i] = Cl ? (int32_t)(Cl[i] & kIdMask) : Cg[i];
    wave_sync();
    lp_dists<G, NCH>(pc, A.f32_base, A.pitch, L.Bi, nR, qv, p, 0.0f, false, L.Bk);
    wave_sync();
    int dummy_min, dummy_in;
    int nr = merge_into_sorted<false>(L.Rk, L.Ri, 0, K, L.Bk, L.Bi, nR, L.Ulo, L.Urank, L.Slo, false, &dummy_min,
                               &dummy_in);
    int pos = nR, batches = 0, n_cut = 0;
    while (pos < nc) {
        const int nb = nc - pos < kappa ? nc - pos : kappa;
        const float thr = L.Rk[nr - 1];
        wave_sync();
        for (int i = lane; i < nb; i += kWave) L.Bi[i] = Cl ? (int32_t)(Cl[pos + i] & kIdMask) : Cg[pos + i];
        wave_sync();
        n_cut += lp_dists<G, NCH>(pc, A.f32_base, A.pitch, L.Bi, nb, qv, p, thr, A.early_abort != 0, L.Bk);
        wave_sync();
        // entries at +inf were aborted: move them out of the merge by id order
        int n_in = 0, min_new;
        nr = merge_into_sorted<false>(L.Rk, L.Ri, nr, K, L.Bk, L.Bi, nb, L.Ulo, L.Urank, L.Slo, false, &min_new, &n_in);
        pos += nb;
        ++batches;
        if (nr - n_in >= m) break;
    }
    wave_sync();
    for (int r = lane; r < A.k_stride; r += kWave) {
        if (r < nr) {
            oid[r] = (int64_t)(L.Ri[r] & kIdMask);
            odist[r] = lp_root(L.Rk[r], p, pc);
        } else {
            oid[r] = -1;
            odist[r] = INFINITY;
        }
    }
    if (lane == 0) {
        st->n_p = pos;
        st->n_cut = n_cut;
        st->batches = batches;
        st->t_end = (uint32_t)wall_clock64();
    }
}

template <int G, int NCH>
__global__ void __launch_bounds__(256) verify_kernel(SearchArgs A) {
    extern __shared__ __attribute__((aligned(16))) char lds_all[];
    const int wave = threadIdx.x / kWave;
    char *lds = lds_all + (size_t)wave * A.lds_wave_bytes;
    const int64_t qi = (int64_t)blockIdx.x * A.waves_per_block + wave;
    if (qi < A.nq) verify_one<G, NCH>(A, qi, lds, A.ncand[qi], A.cand_ids + qi * A.c_stride, nullptr);
}

// Fused walk + verification, one wave per query; with a work counter the
// launch is persistent and waves keep taking queries (in `order` when given)
// until the counter passes nq. C stays in LDS between the two phases; the
// verification's arrays reuse the visited-cache region.
template <int G, int NCH>
__device__ __forceinline__ void verify_call(const SearchArgs &A, int64_t qi, char *lds, int nc,
                                            const uint32_t *Cl) {
    verify_one<G, NCH>(A, qi, lds, nc, nullptr, Cl);
}

// Occupancy target of the fused kernel and VGPRs given to row data in flight.
// Rows of up to 256 dimensions (G <= 16 lanes per row): 5 waves per SIMD
// (<= 96 VGPRs) with 24 VGPRs of row data, for every storage type; the
// verification state makes this kernel larger than the walk, and the extra
// waves pay for the smaller row batches. Measured on the 1M x 128 workload
// (beam 2, 2,048 visited slots): 24 VGPRs (three 8-row steps of 16-bit rows,
// one of FP32 rows) against 32 cut the BF16 launch from 2.37 to 2.28 ms and
// the FP32 one from 3.75 to 3.67 ms (fewer spills in the merge); 16 VGPRs
// give 2.37 ms, and a fourth wave per SIMD with 32 VGPRs 2.65 ms.
// Longer rows (one row per 32 or 64 lanes) keep four rows in flight instead:
// 3 waves with FP32 rows, 4 with 16-bit rows (measured at d = 960).
template <typename T, int G>
constexpr int fused_waves_per_eu() { return G <= 16 ? 5 : (sizeof(T) == 4 ? 3 : 4); }
template <typename T, int G>
constexpr int fused_rb_vgprs() { return G <= 16 ? 24 : (sizeof(T) == 4 ? 64 : 32); }

// BEAM (1 or 2, equal to A.beam) specialises the fused kernel.
template <int G, int NCH, typename T, int BEAM, bool EXT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(fused_waves_per_eu<T, G>(), 8)))
search_kernel(SearchArgs A) {
    extern __shared__ __attribute__((aligned(16))) char lds_all[];
    const int wave = threadIdx.x / kWave;
    char *lds = lds_all + (size_t)wave * A.lds_wave_bytes;
    const WalkLds L = walk_lds(lds, A.ef_cap, A.vis_bits, A.vis_kbits);
    char *vlds = lds + (size_t)A.ef_cap * 8;
    if (A.counter == nullptr) {
        const int64_t k = (int64_t)blockIdx.x * A.waves_per_block + wave;
        const int64_t qi = k < A.nq && A.order ? A.order[k] : k;
        if (k < A.nq) {
            const int nc = walk_one<G, NCH, T, fused_rb_vgprs<T, G>(), false, EXT>(A, qi, lds);
            wave_sync();
            verify_call<G, NCH>(A, qi, vlds, nc, L.Wi);
        }
        return;
    }
    int k = fetch_query(A.counter);
    while ((int64_t)k < A.nq) {
        const int64_t qi = A.order ? A.order[k] : k;
        const int nc = walk_one<G, NCH, T, fused_rb_vgprs<T, G>(), false, EXT>(A, qi, lds);
        wave_sync();
        verify_call<G, NCH>(A, qi, vlds, nc, L.Wi);
        wave_sync();
        k = fetch_query(A.counter);
    }
}

// ------------------------------------------------------------- utilities
// ------------------------------------------------ cost-ordered launch
// Pre-pass: one wave per query runs the descent the walk would run (same
// code, same keys) and records where layer 0 starts. LDS: 64 ids + 64 keys
// per wave.
// Upper-layer rows hold M ids (16 here): 32 VGPRs of rows in flight cover
// one row of FP32 neighbours at d <= 128 (the keys do not depend on how
// many rows are in flight), and 6 waves per SIMD keep more descents going.
template <int G, int NCH, typename T, bool EXT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) descend_kernel(SearchArgs A,
                                                                                                  OrderArgs O) {
    extern __shared__ __attribute__((aligned(16))) char lds_all[];
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    constexpr int kWaveBytes = descend_lds_wave_bytes(EXT);
    int32_t *Uid = reinterpret_cast<int32_t *>(lds_all + (size_t)wave * kWaveBytes);
    float *Uk = reinterpret_cast<float *>(lds_all + (size_t)wave * kWaveBytes + 256);
    float *sqt = reinterpret_cast<float *>(lds_all + (size_t)wave * kWaveBytes + 512);  // EXT only
    const int64_t qi = (int64_t)blockIdx.x * A.waves_per_block + wave;
    if (qi >= A.nq) return;
    const float p = A.p[qi];
    bool finite = true, tiny = false, byte = true;
    for (int j = lane; j < A.d; j += kWave) {
        const float v = A.queries[qi * A.d + j];
        finite = finite && isfinite(v);
        if (EXT) {
            tiny = tiny || (v != 0.0f && fabsf(v) < kL05FastMin);
            byte = byte && is_byte_value(v);
        }
    }
    if (query_bad<EXT>(A, p, A.k[qi], A.ef[qi]) || ballot(!finite) != 0) {
        if (lane == 0) {
            O.entry[qi] = -1;
            O.ekey[qi] = INFINITY;
            O.dnb[qi] = 0;
            O.dist[qi] = -1.0f;  // ordered last: the walk only flags it
        }
        return;
    }
    const int gsel = (p <= A.cutoff) ? 0 : 1;
    const bool lo = gsel == 0;
    float qv[NCH][4];
    load_query<G, NCH>(A.queries + qi * A.d, A.d, qv);
    float kcur;
    int n_b = 0;
    const int root = EXT ? l05_root_mode(A, ballot(tiny) == 0, ballot(!byte) == 0, sqt) : kRootSqrtf;
    const int32_t cur = descend<G, NCH, T, 32, EXT>(A.g[gsel], lo, root, sqt,
                                                    reinterpret_cast<const T *>(A.walk_base), A.pitch, qv, Uid, Uk,
                                                    &kcur, &n_b, A.walk_p);
    if (lane == 0) {
        O.entry[qi] = cur;
        O.ekey[qi] = kcur;
        O.dnb[qi] = n_b;
        // the entry's distance (keys of L2 and L0.5 are its square and root)
        O.dist[qi] = EXT ? (lo ? kcur * kcur : kcur) : (lo ? kcur : sqrtf(kcur));
    }
}

// Dispatch on the row layout: MACRO(G, NCH) for the layout's lane group and
// chunk count.
#define UHNSW_LAYOUT_SWITCH(layout, MACRO) \
    switch (layout) {                      \
        case L8x4x1: MACRO(8, 1); break;   \
        case L8x4x2: MACRO(8, 2); break;   \
        case L8x4x4: MACRO(8, 4); break;   \
        case L16x4x4: MACRO(16, 4); break; \
        case L32x4x4: MACRO(32, 4); break; \
        case L64x4x4: MACRO(64, 4); break; \
        default: return hipErrorInvalidValue; \
    }

}  // namespace uhnsw
