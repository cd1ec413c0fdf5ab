// Device-wide exclusive scan of int64 values (three launches: tile scans, scan of
// tile totals, add).
#include "device.h"
#include "impl.h"

namespace sph {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;

__global__ void __launch_bounds__(kScanThreads) k_tile_scan(const int64_t* in, int64_t* out, int64_t* tile_sum,
                                                           int64_t n) {
  __shared__ int64_t wsum[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int tid = threadIdx.x;
  int64_t v[kScanPer];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    const int64_t idx = base + (int64_t)tid * kScanPer + i;
    v[i] = idx < n ? in[idx] : 0;
    s += v[i];
  }
  int64_t incl = wave_incl_scan(s);
  const int w = tid >> 6;
  if ((tid & 63) == 63) wsum[w] = incl;
  __syncthreads();
  int64_t wpre = 0;
  for (int i = 0; i < w; ++i) wpre += wsum[i];
  int64_t run = wpre + incl - s;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    const int64_t idx = base + (int64_t)tid * kScanPer + i;
    if (idx < n) out[idx] = run;
    run += v[i];
  }
  if (tid == kScanThreads - 1) tile_sum[blockIdx.x] = run;
}

__global__ void __launch_bounds__(64) k_scan_tiles(int64_t* tile_sum, int64_t n_tiles) {
  // single wave, sequential over groups of 64
  int64_t carry = 0;
  for (int64_t b = 0; b < n_tiles; b += 64) {
    const int64_t i = b + threadIdx.x;
    const int64_t v = i < n_tiles ? tile_sum[i] : 0;
    const int64_t incl = wave_incl_scan(v);
    if (i < n_tiles) tile_sum[i] = carry + incl - v;
    carry += __shfl(incl, 63, 64);
  }
}

__global__ void __launch_bounds__(kScanThreads) k_add_tiles(int64_t* out, const int64_t* tile_sum, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int64_t add = tile_sum[blockIdx.x];
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
    const int64_t idx = base + i;
    if (idx < n) out[idx] += add;
  }
}

}  // namespace

void device_exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, DevBuf& tmp, hipStream_t st) {
  if (n <= 0) return;
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  tmp.ensure(sizeof(int64_t) * tiles);
  k_tile_scan<<<dim3((unsigned)tiles), dim3(kScanThreads), 0, st>>>(in, out, tmp.as<int64_t>(), n);
  k_scan_tiles<<<1, 64, 0, st>>>(tmp.as<int64_t>(), tiles);
  k_add_tiles<<<dim3((unsigned)tiles), dim3(kScanThreads), 0, st>>>(out, tmp.as<int64_t>(), n);
  hip_check(hipGetLastError(), "scan launch");
}

}  // namespace sph
