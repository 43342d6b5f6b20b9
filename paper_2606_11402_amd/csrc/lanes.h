// Cross-lane helpers for point groups of P consecutive lanes of a wave64.
// Every lane of the wave is active where these are used and every lane is
// written (row and bank masks 0xF, bound control on), so no old value is
// needed.
//
// A group of P lanes (P = 1, 2, 4, 8, 16 or 32) works on one point; lane r of
// the group owns matrix rows i = p*P + r.  Values owned by another lane of the
// group are read with DPP quad permutes (P <= 4: a modifier of a VALU move,
// no memory pipe) or with ds_swizzle in bit mode (P >= 8: the LDS crossbar,
// inside each half of the wave; no LDS memory is used).
// All selectors are compile-time constants, so the loops that use them are
// unrolled with static_for.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(std::forward<F>(f));
    }
}

// 32-bit value of lane S of this lane's group.
template <int P, int S>
__device__ __forceinline__ int group_bcast_i32(int v) {
    static_assert(P == 1 || P == 2 || P == 4 || P == 8 || P == 16 || P == 32, "group size");
    static_assert(S >= 0 && S < P, "source lane");
    if constexpr (P == 1) {
        return v;
    } else if constexpr (P == 2) {
        // pairs (0,1), (2,3) inside each quad
        constexpr int ctrl = (S) | (S << 2) | ((2 + S) << 4) | ((2 + S) << 6);
        return __builtin_amdgcn_mov_dpp(v, ctrl, 0xF, 0xF, true);
    } else if constexpr (P == 4) {
        constexpr int ctrl = S | (S << 2) | (S << 4) | (S << 6);
        return __builtin_amdgcn_mov_dpp(v, ctrl, 0xF, 0xF, true);
    } else {
        // bit mode: lane' = (lane & and_mask) | or_mask, within 32 lanes; the
        // and_mask keeps the bits above the group (group of 8: bits 3-4,
        // group of 16: bit 4, group of 32: none)
        constexpr int and_mask = P == 8 ? 0x18 : (P == 16 ? 0x10 : 0x00);
        constexpr int pattern = and_mask | (S << 5);
        return __builtin_amdgcn_ds_swizzle(v, pattern);
    }
}

// 32-bit value of the lane whose index differs by X (X in {1, 2, 4, 8, 16,
// 32}; 32 crosses the halves of the wave, through ds_bpermute).
template <int X>
__device__ __forceinline__ int group_xor_i32(int v) {
    if constexpr (X == 1) {
        return __builtin_amdgcn_mov_dpp(v, 1 | (0 << 2) | (3 << 4) | (2 << 6), 0xF, 0xF, true);
    } else if constexpr (X == 2) {
        return __builtin_amdgcn_mov_dpp(v, 2 | (3 << 2) | (0 << 4) | (1 << 6), 0xF, 0xF, true);
    } else if constexpr (X == 32) {
        return __shfl_xor(v, 32, 64);
    } else {
        static_assert(X == 4 || X == 8 || X == 16, "xor distance");
        return __builtin_amdgcn_ds_swizzle(v, 0x1F | (X << 10));
    }
}

template <int P, int S>
__device__ __forceinline__ float group_bcast(float v) {
    return __int_as_float(group_bcast_i32<P, S>(__float_as_int(v)));
}

template <int P, int S>
__device__ __forceinline__ double group_bcast(double v) {
    const int64_t u = __double_as_longlong(v);
    const int lo = group_bcast_i32<P, S>((int)(u & 0xffffffff));
    const int hi = group_bcast_i32<P, S>((int)(u >> 32));
    return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

template <int P, int S>
__device__ __forceinline__ int group_bcast(int v) {
    return group_bcast_i32<P, S>(v);
}

template <int X>
__device__ __forceinline__ float group_xor(float v) {
    return __int_as_float(group_xor_i32<X>(__float_as_int(v)));
}

template <int X>
__device__ __forceinline__ double group_xor(double v) {
    const int64_t u = __double_as_longlong(v);
    const int lo = group_xor_i32<X>((int)(u & 0xffffffff));
    const int hi = group_xor_i32<X>((int)(u >> 32));
    return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// Sum over the P lanes of the group; every lane receives the same bits
// (pairwise butterfly, each addition commutative).
template <int P, typename T>
__device__ __forceinline__ T group_sum(T v) {
    if constexpr (P >= 2) v = v + group_xor<1>(v);
    if constexpr (P >= 4) v = v + group_xor<2>(v);
    if constexpr (P >= 8) v = v + group_xor<4>(v);
    if constexpr (P >= 16) v = v + group_xor<8>(v);
    if constexpr (P >= 32) v = v + group_xor<16>(v);
    if constexpr (P >= 64) v = v + group_xor<32>(v);
    return v;
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip; map the
// hardware block index so that each XCD works on one contiguous range of
// logical blocks (neighbouring tiles share that XCD's L2).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
    const int64_t per = nb >> 3, rem = nb & 7;
    const int64_t xcd = b & 7, idx = b >> 3;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}
