// Device helpers: wave/work-group scans and the in-LDS radix sort of a ray's knot keys.
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

// inclusive scan of a uint32 over the 64 lanes of a wave with DPP lane moves (no LDS):
// Hillis-Steele within each row of 16 lanes, then row 0's total into row 1 and row 2's into row 3
// (row_bcast:15), then the total of rows 0-1 into rows 2-3 (row_bcast:31)
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
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

// Stable LSD radix sort of a[0..n) by bits [lo_bit, lo_bit + nbits) with 4-bit digits, by all
// NT threads of the work-group, n <= 1023 NT.  Thread t owns the contiguous block [t m, (t+1) m),
// m = ceil(n / NT) rounded up to odd (an odd stride of 8-byte elements spreads a wave's reads over
// the LDS banks).  Per pass a thread loads its keys in batches of 16 into registers and counts
// its digits in packed 16-bit fields; a wave scan of the packed fields gives each lane its rank
// among the wave's equal digits, and a 16 x (NT/64) table in LDS gives each (wave, digit) its
// base, so the scatter keeps equal digits in order with no read-modify-write of shared counters.
// tab: 32 * (NT / 64) uint32 of LDS.  The result ends in `a`; with PAD_OUT it is stored with one
// unused slot after every 16 elements (element i at i + i / 16; a and tmp then hold
// n + n / 16 + 1 elements).  Caller guarantees a barrier before; ends with a barrier.
template <int NT, bool PAD_OUT>
__device__ __forceinline__ void radix_sort_u64(uint64_t* a, uint64_t* tmp, int n, int lo_bit, int nbits, uint32_t* tab, int tid) {
  constexpr int W = NT / 64;
  constexpr int E = (16 * W + 63) / 64;  // table entries per lane of the scanning wave
  constexpr int MB = 16;
  uint32_t* cnt = tab;             // [W][16] digit counts per wave
  uint32_t* wbase = tab + 16 * W;  // [W][16] first output slot per (wave, digit)
  const int m = ((n + NT - 1) / NT) | 1;
  const int b0 = min(tid * m, n), b1 = min(b0 + m, n);
  const int w = tid >> 6, lane = tid & 63;
  uint64_t* src = a;
  uint64_t* dst = tmp;
  for (int shift = lo_bit; shift < lo_bit + nbits; shift += 4) {
    const bool last = shift + 4 >= lo_bit + nbits;
    uint64_t c[4] = {0, 0, 0, 0};  // 16 counters of 16 bits
    for (int i0 = b0; i0 < b1; i0 += MB) {
      uint64_t kv[MB];
#pragma unroll
      for (int k = 0; k < MB; ++k) kv[k] = (i0 + k < b1) ? src[i0 + k] : 0ull;
#pragma unroll
      for (int k = 0; k < MB; ++k) {
        const uint32_t d = (uint32_t)(kv[k] >> shift) & 15u;
        const uint64_t inc = (i0 + k < b1) ? (1ull << (16 * (d & 3))) : 0ull;
        const uint32_t q = d >> 2;
        c[0] += (q == 0) ? inc : 0ull;
        c[1] += (q == 1) ? inc : 0ull;
        c[2] += (q == 2) ? inc : 0ull;
        c[3] += (q == 3) ? inc : 0ull;
      }
    }
    // rank of this lane's first key of each digit among the wave's keys of that digit (the packed
    // fields stay below 2^16, so the two 32-bit halves scan independently)
    uint64_t pre[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t il = wave_incl_scan_u32((uint32_t)c[q]);
      const uint32_t ih = wave_incl_scan_u32((uint32_t)(c[q] >> 32));
      const uint64_t incl = ((uint64_t)ih << 32) | il;
      pre[q] = incl - c[q];
      if (lane == 63) {
#pragma unroll
        for (int f = 0; f < 4; ++f) cnt[w * 16 + 4 * q + f] = (uint32_t)((incl >> (16 * f)) & 0xffffu);
      }
    }
    __syncthreads();
    if (w == 0) {
      // entry (wave ww, digit d) = all keys of smaller digits plus this digit's keys of earlier
      // waves: one exclusive scan over the entries in digit-major order e = d * W + ww, E
      // consecutive entries per lane
      uint32_t x[E], sum = 0;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int e = lane * E + j, d = e / W, ww = e % W;
        x[j] = (e < 16 * W) ? cnt[ww * 16 + d] : 0u;
        sum += x[j];
      }
      uint32_t run = wave_incl_scan_u32(sum) - sum;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int e = lane * E + j, d = e / W, ww = e % W;
        if (e < 16 * W) wbase[ww * 16 + d] = run;
        run += x[j];
      }
    }
    __syncthreads();
    for (int i0 = b0; i0 < b1; i0 += MB) {
      uint64_t kv[MB];
#pragma unroll
      for (int k = 0; k < MB; ++k) kv[k] = (i0 + k < b1) ? src[i0 + k] : 0ull;
#pragma unroll
      for (int k = 0; k < MB; ++k) {
        if (i0 + k < b1) {
          const uint32_t d = (uint32_t)(kv[k] >> shift) & 15u;
          const uint32_t q = d >> 2, sh = 16 * (d & 3);
          const uint64_t pq = (q == 0) ? pre[0] : ((q == 1) ? pre[1] : ((q == 2) ? pre[2] : pre[3]));
          const uint32_t p = min(wbase[w * 16 + d] + (uint32_t)((pq >> sh) & 0xffffu), (uint32_t)(n - 1));
          const uint64_t inc = 1ull << sh;
          pre[0] += (q == 0) ? inc : 0ull;
          pre[1] += (q == 1) ? inc : 0ull;
          pre[2] += (q == 2) ? inc : 0ull;
          pre[3] += (q == 3) ? inc : 0ull;
          dst[(PAD_OUT && last) ? p + (p >> 4) : p] = kv[k];
        }
      }
    }
    __syncthreads();
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  if (src != a) {
    const int np = PAD_OUT ? n + (n >> 4) : n;
    for (int i = tid; i < np; i += NT) a[i] = src[i];
    __syncthreads();
  }
}

// Stable LSD radix sort of a[0..n) by bits [lo_bit, lo_bit + nbits) with 8-bit digits (the last
// one narrower when nbits is not a multiple of 8), by the NT threads of the work-group.  Wave w
// owns the contiguous segment [w s, (w + 1) s) of each pass's source, s = ceil(n / W).  The digit
// counts of a pass are kept per (wave, digit): the first pass counts them directly, every pass
// counts the next pass's while it moves the keys (a key written to slot p belongs to wave p / s
// next time).  Per pass one wave turns the W x 256 counts into first output slots by an exclusive
// scan in digit-major order (all keys of smaller digits, then this digit's keys of earlier waves);
// each wave then moves its segment in rounds of 64 keys, a key's rank among the round's equal
// digits coming from a match over the digit's bits (one ballot per bit) and the digit's slot
// advancing by the round's count, so no work-group barrier is needed inside the pass and equal
// digits keep their order; n <= 2^16 W - W (a wave's segment of counts fits 16 bits).  tab: 384 * W
// uint32 of LDS.  The result ends in `a`; with PAD_OUT
// it is stored with one unused slot after every 16 elements (element i at i + i / 16; a and tmp
// then hold n + n / 16 + 1 elements).  Caller guarantees a barrier before; ends with a barrier.
template <int NT, bool PAD_OUT>
__device__ __forceinline__ void radix_sort_u64_d8(uint64_t* a, uint64_t* tmp, int n, int lo_bit, int nbits,
                                                  uint32_t* tab, int tid) {
  constexpr int W = NT / 64;
  constexpr int E = 256 * W / 64;  // scan entries per lane
  const int w = tid >> 6, lane = tid & 63;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int seg = (n + W - 1) / W;
  const int s0 = min(w * seg, n), s1 = min(s0 + seg, n);
  uint32_t* cur = tab;             // [W][256] this pass's first output slots
  uint32_t* cnt = tab + 256 * W;   // [W][128] digit counts, two 16-bit fields per word (a wave's
                                   // segment holds fewer than 2^16 keys)
  uint64_t* src = a;
  uint64_t* dst = tmp;
  for (int i = tid; i < 128 * W; i += NT) cnt[i] = 0u;
  __syncthreads();
  {
    const uint32_t mask = (1u << min(8, nbits)) - 1u;
    for (int i = s0 + lane; i < s1; i += 64) {
      const uint32_t d = (uint32_t)(src[i] >> lo_bit) & mask;
      atomicAdd(&cnt[w * 128 + (d >> 1)], 1u << (16 * (d & 1u)));
    }
  }
  for (int shift = lo_bit; shift < lo_bit + nbits; shift += 8) {
    const int bits = min(8, lo_bit + nbits - shift);
    const uint32_t mask = (1u << bits) - 1u;
    const bool last = shift + 8 >= lo_bit + nbits;
    const uint32_t mask_n = last ? 0u : (1u << min(8, lo_bit + nbits - shift - 8)) - 1u;
    __syncthreads();
    if (w == 0) {
      // entry e = d * W + ww (digit-major), E consecutive entries per lane; the counts are read,
      // then cleared for the counts of the next pass, then turned into slots
      uint32_t x[E], sum = 0;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int e = lane * E + j, d = e / W, ww = e % W;
        x[j] = (cnt[ww * 128 + (d >> 1)] >> (16 * (d & 1))) & 0xffffu;
        sum += x[j];
      }
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int e = lane * E + j, d = e / W, ww = e % W;
        cnt[ww * 128 + (d >> 1)] = 0u;
      }
      uint32_t run = wave_incl_scan_u32(sum) - sum;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int e = lane * E + j, d = e / W, ww = e % W;
        cur[ww * 256 + d] = run;
        run += x[j];
      }
    }
    __syncthreads();
    uint32_t* mine = cur + w * 256;
    for (int i0 = s0; i0 < s1; i0 += 64) {
      const int i = i0 + lane;
      const bool valid = i < s1;
      const uint64_t k = valid ? src[i] : 0ull;
      const uint32_t d = (uint32_t)(k >> shift) & mask;
      uint64_t m = __ballot(valid);
      for (int b = 0; b < bits; ++b) {
        const uint64_t bal = __ballot((d >> b) & 1u);
        m &= ((d >> b) & 1u) ? bal : ~bal;
      }
      const uint32_t rank = (uint32_t)__popcll(m & lt);
      const uint32_t c = valid ? mine[d] : 0u;
      __builtin_amdgcn_wave_barrier();
      if (valid) {
        const uint32_t p = min(c + rank, (uint32_t)(n - 1));  // (always below n; kept in bounds regardless)
        dst[(PAD_OUT && last) ? p + (p >> 4) : p] = k;
        if (rank == 0) mine[d] = c + (uint32_t)__popcll(m);
        if (!last) {
          const uint32_t dn = (uint32_t)(k >> (shift + 8)) & mask_n;
          atomicAdd(&cnt[(p / (uint32_t)seg) * 128 + (dn >> 1)], 1u << (16 * (dn & 1u)));
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  __syncthreads();
  if (src != a) {
    const int np = PAD_OUT ? n + (n >> 4) : n;
    for (int i = tid; i < np; i += NT) a[i] = src[i];
    __syncthreads();
  }
}

}  // namespace sph
