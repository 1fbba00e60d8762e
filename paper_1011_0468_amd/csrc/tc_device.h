// Device-side helpers for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// bits of lanes strictly below this lane
__device__ __forceinline__ uint64_t lanes_below() {
    const int l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint64_t ballot64(int pred) { return __ballot(pred); }

// inclusive wave scan (sum)
template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T o = __shfl_up(v, d, 64);
        if (__lane_id() >= d) v += o;
    }
    return v;
}

// The same for 32-bit integers with DPP lane moves (no LDS crossbar round
// trips): prefixes within each row of 16 lanes by shifts of 1, 2, 4 and 8,
// then the last lane of row 0 is added to row 1 and that of row 2 to row 3,
// and the last lane of row 1 to rows 2 and 3.  Whole wave.
__device__ __forceinline__ int32_t wave_inclusive_sum(int32_t v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        T o = __shfl_xor(v, d, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Exclusive scan over a block of NT threads (NT multiple of 64, <= 1024).
// `tmp` must hold NT/64 + 1 elements of LDS.  Returns the exclusive prefix of
// this thread and writes the block total to *total.
template <int NT, typename T>
__device__ __forceinline__ T block_exclusive_sum(T v, T* tmp, T* total) {
    constexpr int NW = NT / 64;
    const int w = threadIdx.x >> 6;
    T inc = wave_inclusive_sum(v);
    if (__lane_id() == 63) tmp[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = 0;
        for (int i = 0; i < NW; ++i) { T t = tmp[i]; tmp[i] = acc; acc += t; }
        tmp[NW] = acc;
    }
    __syncthreads();
    T r = tmp[w] + inc - v;
    *total = tmp[NW];
    __syncthreads();
    return r;
}

// SplitMix64 output function (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

// Keep decision of the undirected edge {u,v}: section 3.1's independent coin,
// realised as a hash of (min, max) salted by the seed.
__device__ __forceinline__ bool edge_kept(uint32_t u, uint32_t v, uint64_t salt, uint64_t thr) {
    const uint64_t lo = u < v ? u : v;
    const uint64_t hi = u < v ? v : u;
    const uint64_t h = mix64(mix64((lo << 32) | hi) ^ salt);
    return (h >> 11) < thr;
}

// (deg, id) rank order
__device__ __forceinline__ bool rank_below(int32_t du, int32_t u, int32_t dv, int32_t v) {
    return du < dv || (du == dv && u < v);
}

}  // namespace tc
