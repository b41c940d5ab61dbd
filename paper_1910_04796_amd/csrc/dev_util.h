// dev_util.h -- wave64 / workgroup primitives used by the library's kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bsmm {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Orders the LDS traffic of one wavefront: every LDS access issued before it
// has completed, and the compiler moves no memory access across it.  Lanes
// of a wave execute in lockstep, so this is all a wave-private exchange
// through LDS needs.
__device__ __forceinline__ void wave_lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

template <class T> __device__ __forceinline__ T wave_inclusive_scan(T v) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T u = __shfl_up(v, d, kWave);
        if (l >= d) v += u;
    }
    return v;
}

template <class T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

template <class T> __device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        T u = __shfl_xor(v, d, kWave);
        v = u > v ? u : v;
    }
    return v;
}

// Sum over a workgroup of up to 16 waves; every thread gets the result.
template <class T> __device__ __forceinline__ T block_sum(T v, T *lds16) {
    v = wave_sum(v);
    const int w = wave_id(), nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (lane_id() == 0) lds16[w] = v;
    __syncthreads();
    T t = 0;
    for (int i = 0; i < nw; ++i) t += lds16[i];
    __syncthreads();
    return t;
}

// Exclusive scan over a workgroup of up to 16 waves; *total gets the sum.
template <class T> __device__ __forceinline__ T block_exclusive_scan(T v, T *lds16, T *total) {
    T inc = wave_inclusive_scan(v);
    const int w = wave_id(), nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (lane_id() == kWave - 1) lds16[w] = inc;
    __syncthreads();
    T base = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < w) base += lds16[i];
        tot += lds16[i];
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

// Floor division of small non-negative integers (e < 2^20, 1 <= d < 2^12) by
// a float reciprocal (quotient error below 1/4) followed by an exact
// one-step correction.
__device__ __forceinline__ int divmod_small(int e, int d, float rcp, int *rem) {
    int q = (int)((float)e * rcp);
    int r = e - q * d;
    if (r < 0) { q -= 1; r += d; }
    else if (r >= d) { q += 1; r -= d; }
    *rem = r;
    return q;
}

}  // namespace bsmm
