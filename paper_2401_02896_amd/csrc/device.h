// Device helpers: wave/work-group scans and an in-LDS bitonic sort.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sph {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// inclusive scan over the 64 lanes of a wave
template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int l = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T n = __shfl_up(v, o, 64);
    if (l >= o) v += n;
  }
  return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    T n = __shfl_xor(v, o, 64);
    v = v > n ? v : n;
  }
  return v;
}

__device__ __forceinline__ int next_pow2(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Ascending sort of a[0..n) (any n) by all threads of the work-group, using the
// bitonic network with the "flip" first stage of every merge so that the
// missing elements n..next_pow2(n) behave as +infinity and never move.
// Caller guarantees a barrier before (data ready); ends with a barrier.
template <class T>
__device__ void bitonic_sort(T* a, int n, int tid, int nthreads) {
  const int np2 = next_pow2(n);
  const int half = np2 >> 1;
  for (int k = 2; k <= np2; k <<= 1) {
    const int hk = k >> 1;
    for (int c = tid; c < half; c += nthreads) {
      const int blk = c / hk, j = c - blk * hk;
      const int lo = blk * k + j, hi = blk * k + k - 1 - j;
      if (hi < n) {
        T x = a[lo], y = a[hi];
        if (y < x) {
          a[lo] = y;
          a[hi] = x;
        }
      }
    }
    __syncthreads();
    for (int s = hk >> 1; s >= 1; s >>= 1) {
      for (int c = tid; c < half; c += nthreads) {
        const int blk = c / s, j = c - blk * s;
        const int lo = blk * 2 * s + j, hi = lo + s;
        if (hi < n) {
          T x = a[lo], y = a[hi];
          if (y < x) {
            a[lo] = y;
            a[hi] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

}  // namespace sph
