// Device helpers shared by the gfx950 kernels: packed keys and wave64 /
// workgroup reductions.  Included by .hip sources only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dgs_internal.h"

namespace dgs {
namespace dev {

// ---- packed keys -----------------------------------------------------------
// key(g, idx): unsigned order == (g ascending, idx descending).  Key 0 is
// "no candidate": a real gain is > -2^31, so its biased high word is > 0.
__device__ __forceinline__ u64 mk_key(int g, int idx) {
    return ((u64)((uint32_t)g ^ 0x80000000u) << 32) | (u64)(~(uint32_t)idx);
}
__device__ __forceinline__ int key_gain(u64 k) { return (int)((uint32_t)(k >> 32) ^ 0x80000000u); }
__device__ __forceinline__ int key_index(u64 k) { return (int)(~(uint32_t)k); }

__device__ __forceinline__ u64 umax64(u64 a, u64 b) { return a > b ? a : b; }
__device__ __forceinline__ u64 umin64(u64 a, u64 b) { return a < b ? a : b; }

// ---- wave64 lane exchanges on the VALU (no LDS round trip) -----------------
// xor_lanes<J>(v) is the value of lane (lane ^ J): J = 1, 2 are DPP quad
// permutes, J = 8 a DPP rotate by 8 within a 16-lane row, J = 4 one of the
// two DPP rotates by 4 / 12 (picked by applying the same rotate to the lane
// index, so the result does not depend on the rotate's direction), and
// J = 16, 32 the gfx950 permlane swaps.  Every lane of the wave must be
// active.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}

template <int J>
__device__ __forceinline__ uint32_t xor_lanes(uint32_t v) {
    if constexpr (J == 1) {
        return dpp32<0xB1>(v);  // quad_perm [1, 0, 3, 2]
    } else if constexpr (J == 2) {
        return dpp32<0x4E>(v);  // quad_perm [2, 3, 0, 1]
    } else if constexpr (J == 4) {
        const uint32_t lane = threadIdx.x & 63;
        const uint32_t a = dpp32<0x124>(v), b = dpp32<0x12C>(v);  // row_ror 4, row_ror 12
        return dpp32<0x124>(lane) == (lane ^ 4u) ? a : b;
    } else if constexpr (J == 8) {
        return dpp32<0x128>(v);  // row_ror 8
    } else if constexpr (J == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (threadIdx.x & 16) ? r[0] : r[1];
    } else {
        static_assert(J == 32, "lane distance");
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (threadIdx.x & 32) ? r[0] : r[1];
    }
}

template <int J>
__device__ __forceinline__ u64 xor_lanes64(u64 v) {
    return ((u64)xor_lanes<J>((uint32_t)(v >> 32)) << 32) | (u64)xor_lanes<J>((uint32_t)v);
}

// The value of lane (lane ^ mask).  In unrolled loops the mask is a
// constant and the switch folds to one xor_lanes; other masks go through
// ds_bpermute.
__device__ __forceinline__ u64 shfl_xor64(u64 v, int mask) {
    switch (mask) {
        case 1: return xor_lanes64<1>(v);
        case 2: return xor_lanes64<2>(v);
        case 4: return xor_lanes64<4>(v);
        case 8: return xor_lanes64<8>(v);
        case 16: return xor_lanes64<16>(v);
        case 32: return xor_lanes64<32>(v);
        default: break;
    }
    const int lo = __shfl_xor((int)(uint32_t)v, mask, 64);
    const int hi = __shfl_xor((int)(uint32_t)(v >> 32), mask, 64);
    return ((u64)(uint32_t)hi << 32) | (u64)(uint32_t)lo;
}

// Maximum over the wave, every lane gets it (all lanes active).
template <int M = 32>
__device__ __forceinline__ u64 wave_max64(u64 v) {
    v = umax64(v, xor_lanes64<M>(v));
    if constexpr (M > 1) return wave_max64<M / 2>(v);
    return v;
}

// Lane `lane`'s value (lane uniform across the wave), through SGPRs.
__device__ __forceinline__ u64 readlane64(u64 v, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((u64)hi << 32) | lo;
}

// The value of lane 63 - lane (row mirror, then the 16- and 32-lane swaps).
__device__ __forceinline__ u64 reverse_lanes64(u64 v) {
    const uint32_t lo = xor_lanes<32>(xor_lanes<16>(dpp32<0x140>((uint32_t)v)));
    const uint32_t hi = xor_lanes<32>(xor_lanes<16>(dpp32<0x140>((uint32_t)(v >> 32))));
    return ((u64)hi << 32) | lo;
}

// Top-2 of a set of unique keys (0 = empty slot).
__device__ __forceinline__ void top2_push(u64 &b1, u64 &b2, u64 k) {
    u64 lo = umin64(b1, k);
    b1 = umax64(b1, k);
    b2 = umax64(b2, lo);
}
__device__ __forceinline__ void top2_merge(u64 &a1, u64 &a2, u64 b1, u64 b2) {
    u64 lo = umin64(a1, b1);
    a1 = umax64(a1, b1);
    a2 = umax64(umax64(a2, b2), lo);
}

// Top-2 with the partner agent of the best entry.
struct Best2 {
    u64 k1, k2;
    int c1;
};
__device__ __forceinline__ void best2_push(Best2 &a, u64 k, int c) {
    if (k > a.k1) {
        a.k2 = a.k1;
        a.k1 = k;
        a.c1 = c;
    } else {
        a.k2 = umax64(a.k2, k);
    }
}
__device__ __forceinline__ void best2_merge(Best2 &a, u64 k1, u64 k2, int c1) {
    if (k1 > a.k1) {
        a.k2 = umax64(a.k1, k2);
        a.k1 = k1;
        a.c1 = c1;
    } else {
        a.k2 = umax64(a.k2, k1);
    }
}

// Triangular index p -> (I, K), I <= K < nb, row-major over I.
__device__ __forceinline__ void pair_of(long long p, int nb, int &I, int &K) {
    // pairs before row I: I*nb - I*(I-1)/2
    const double b = 2.0 * nb + 1.0;
    int i = (int)((b - sqrt(b * b - 8.0 * (double)p)) * 0.5);
    if (i < 0) i = 0;
    if (i > nb - 1) i = nb - 1;
    auto start = [&](int r) { return (long long)r * nb - (long long)r * (r - 1) / 2; };
    while (i > 0 && start(i) > p) --i;
    while (i + 1 < nb && start(i + 1) <= p) ++i;
    I = i;
    K = i + (int)(p - start(i));
}

// Wave reductions over the lane distances M, M / 2, ..., 1 as template
// arguments: every exchange is a VALU lane permute whatever the compiler's
// unrolling does (a distance known only at run time goes through the LDS).
// Every lane of the wave must be active; every lane gets the result.
template <int M = 32>
__device__ __forceinline__ void wave_top2(u64 &b1, u64 &b2) {
    top2_merge(b1, b2, xor_lanes64<M>(b1), xor_lanes64<M>(b2));
    if constexpr (M > 1) wave_top2<M / 2>(b1, b2);
}
template <int M = 32>
__device__ __forceinline__ void wave_best2(Best2 &a) {
    const u64 o1 = xor_lanes64<M>(a.k1), o2 = xor_lanes64<M>(a.k2);
    const int oc = (int)xor_lanes<M>((uint32_t)a.c1);
    best2_merge(a, o1, o2, oc);
    if constexpr (M > 1) wave_best2<M / 2>(a);
}

// Block reductions over BLOCK threads (BLOCK a multiple of 64).  `lds`
// holds at least 3 * BLOCK / 64 u64.  Every thread gets the result.
template <int BLOCK>
__device__ u64 block_max(u64 v, u64 *lds) {
    v = wave_max64(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    u64 r = lds[0];
#pragma unroll
    for (int i = 1; i < BLOCK / 64; ++i) r = umax64(r, lds[i]);
    return r;
}

template <int BLOCK>
__device__ void block_top2(u64 &b1, u64 &b2, u64 *lds) {
    wave_top2(b1, b2);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        lds[2 * w] = b1;
        lds[2 * w + 1] = b2;
    }
    __syncthreads();
    b1 = lds[0];
    b2 = lds[1];
#pragma unroll
    for (int i = 1; i < BLOCK / 64; ++i) top2_merge(b1, b2, lds[2 * i], lds[2 * i + 1]);
}

template <int BLOCK>
__device__ void block_best2(Best2 &a, u64 *lds) {
    wave_best2(a);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        lds[3 * w] = a.k1;
        lds[3 * w + 1] = a.k2;
        lds[3 * w + 2] = (u64)(uint32_t)a.c1;
    }
    __syncthreads();
    a.k1 = lds[0];
    a.k2 = lds[1];
    a.c1 = (int)(uint32_t)lds[2];
#pragma unroll
    for (int i = 1; i < BLOCK / 64; ++i) best2_merge(a, lds[3 * i], lds[3 * i + 1], (int)(uint32_t)lds[3 * i + 2]);
}


}  // namespace dev
}  // namespace dgs
