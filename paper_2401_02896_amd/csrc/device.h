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

// Exclusive prefix sum of one int64 per thread over the NT threads of the work-group (in thread
// order); *total receives the sum.  wtot: NT / 64 int64 of LDS.  Starts and ends with a barrier
// on wtot, so it can be called back to back.
template <int NT>
__device__ int64_t block_excl_scan_i64(int64_t v, int64_t* wtot, int tid, int64_t* total) {
  const int64_t incl = wave_incl_scan<long>((long)v);
  const int w = tid >> 6;
  __syncthreads();
  if ((tid & 63) == 63) wtot[w] = incl;
  __syncthreads();
  int64_t pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    const int64_t x = wtot[i];
    pre += (i < w) ? x : 0;
    tot += x;
  }
  *total = tot;
  __syncthreads();
  return pre + incl - v;
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

// Stable LSD radix sort of a[0..n) by bits [lo_bit, lo_bit + nbits) with 4-bit digits, by all
// NT threads of the work-group.  Thread t owns the contiguous block [t m, (t+1) m), m = ceil(n/NT),
// counts its digits in packed 16-bit register fields, and scatters its block in order after a
// work-group scan of the (digit, thread) counts, so equal digits keep their order.
// tmp: n elements of scratch; hist: 16 * NT uint32 (LDS); wsum: NT / 64 + 1 uint32 (LDS).
// The result ends in `a`.  Caller guarantees a barrier before; ends with a barrier.
template <int NT>
__device__ void radix_sort_u64(uint64_t* a, uint64_t* tmp, int n, int lo_bit, int nbits, uint32_t* hist,
                               uint32_t* wsum, int tid) {
  const int m = (n + NT - 1) / NT;
  const int b0 = min(tid * m, n), b1 = min(b0 + m, n);
  uint64_t* src = a;
  uint64_t* dst = tmp;
  for (int shift = lo_bit; shift < lo_bit + nbits; shift += 4) {
    uint64_t c[4] = {0, 0, 0, 0};  // 16 counters of 16 bits
    for (int i = b0; i < b1; ++i) {
      const uint32_t d = (uint32_t)(src[i] >> shift) & 15u;
      const uint64_t inc = 1ull << (16 * (d & 3));
      const uint32_t q = d >> 2;
      c[0] += (q == 0) ? inc : 0ull;
      c[1] += (q == 1) ? inc : 0ull;
      c[2] += (q == 2) ? inc : 0ull;
      c[3] += (q == 3) ? inc : 0ull;
    }
#pragma unroll
    for (int d = 0; d < 16; ++d) hist[d * NT + tid] = (uint32_t)((c[d >> 2] >> (16 * (d & 3))) & 0xffffu);
    __syncthreads();
    // exclusive scan of hist[0 .. 16 NT) in memory order: thread t takes entries [16 t, 16 t + 16)
    uint32_t loc[16];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      loc[k] = s;
      s += hist[tid * 16 + k];
    }
    const uint32_t incl = wave_incl_scan(s);
    const int w = tid >> 6;
    if ((tid & 63) == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t pre = incl - s;
    for (int i = 0; i < w; ++i) pre += wsum[i];
#pragma unroll
    for (int k = 0; k < 16; ++k) hist[tid * 16 + k] = loc[k] + pre;
    __syncthreads();
    for (int i = b0; i < b1; ++i) {
      const uint64_t v = src[i];
      const uint32_t d = (uint32_t)(v >> shift) & 15u;
      const uint32_t p = hist[d * NT + tid];
      hist[d * NT + tid] = p + 1;
      dst[p] = v;
    }
    __syncthreads();
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  if (src != a) {
    for (int i = tid; i < n; i += NT) a[i] = src[i];
    __syncthreads();
  }
}

}  // namespace sph
