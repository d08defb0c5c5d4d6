// Wave64 / workgroup primitives shared by the kernel translation units.
#pragma once

#include "common.h"

namespace kt {

// New position q of element e (kept), or ~q (dropped, q kept elements before it).
__device__ __forceinline__ int32_t keep_rank(const KeepWord* __restrict__ kw, int32_t e) {
    const KeepWord k = kw[e >> 6];
    const int b = e & 63;
    const int32_t q = k.pref + __popcll(k.bits & ((1ull << b) - 1ull));
    return ((k.bits >> b) & 1ull) ? q : ~q;
}

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o);
        if (lane >= o) v += u;
    }
    return v;
}

// Exclusive prefix of 0/1 `flag` over a workgroup of NT threads (ballot +
// mbcnt inside each wave, wave totals through LDS `s_wave[NT/64]`).
template <int NT>
__device__ __forceinline__ int block_excl_flag(bool flag, int* s_wave, int& total) {
    const uint64_t bal = __ballot(flag);
    const int w = threadIdx.x >> 6;
    const int pre = (int)lanes_below(bal);
    if (__lane_id() == 0) s_wave[w] = __popcll(bal);
    __syncthreads();
    int wpre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        const int c = s_wave[i];
        wpre += i < w ? c : 0;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return wpre + pre;
}

// Exclusive prefix of an int over a workgroup of NT threads.
template <int NT>
__device__ __forceinline__ int block_excl_sum(int v, int* s_wave, int& total) {
    const int inc = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 63) s_wave[w] = inc;
    __syncthreads();
    int wpre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        const int c = s_wave[i];
        wpre += i < w ? c : 0;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return wpre + inc - v;
}

template <int NT>
__device__ __forceinline__ int block_sum(int v, int* s_wave) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 0) s_wave[w] = v;
    __syncthreads();
    int tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) tot += s_wave[i];
    __syncthreads();
    return tot;
}

// 64-bit versions of the workgroup exclusive sum and total.
template <int NT>
__device__ __forceinline__ long long block_excl_sum64(long long v, long long* s_wave, long long& total) {
    const int lane = __lane_id();
    long long inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long u = __shfl_up(inc, o);
        if (lane >= o) inc += u;
    }
    const int w = threadIdx.x >> 6;
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    long long wpre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        const long long c = s_wave[i];
        wpre += i < w ? c : 0;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return wpre + inc - v;
}

template <int NT>
__device__ __forceinline__ long long block_sum64(long long v, long long* s_wave) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 0) s_wave[w] = v;
    __syncthreads();
    long long tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) tot += s_wave[i];
    __syncthreads();
    return tot;
}

static inline unsigned grid_for(int64_t items, int per_block = kBlock) {
    int64_t g = (items + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g);
}

// First index in the ascending list a[0, len) whose value is >= x.
__device__ __forceinline__ int32_t lower_bound_i32(const int32_t* __restrict__ a, int32_t len, int32_t x) {
    int32_t lo = 0;
    while (len > 0) {
        const int32_t half = len >> 1;
        if (a[lo + half] < x) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

}  // namespace kt
