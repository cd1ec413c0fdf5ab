// Particle index build: validation, multi-level Morton grid, a_max bound and
// representative attributes (the data analysis of Sec. 4.4).
//
// Grid definition (the paper leaves the search for a particle's relevant rays
// open; Sec. 2, first pass): c_0 is the smallest power of two >= min(q h),
// doubled until level 0 has at most 2^24 cells and 2^19 per axis; a particle
// lives on the smallest level l with q h <= c_l = c_0 2^l, in the cell
// floor((x - lo) * (1 / c_l)) (float64, lo = per-axis minimum).  Particles are
// ordered by (level, Morton code of the cell, input index) with a stable LSD
// radix sort; each cell's particles are then contiguous.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "device.h"
#include "impl.h"

namespace sph {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t f2ord(float f) {
  uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ inline float ord2f(uint32_t o) {
  uint32_t b = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  float f;
  memcpy(&f, &b, 4);
  return f;
}

// mins[0..3] = min x, y, z, h; maxs[0..3] = max x, y, z, h (ordered-int encoding)
__global__ void __launch_bounds__(kThreads) k_validate_bounds(const float* xyz, const float* h, const float* val,
                                                              int64_t n, uint32_t* mins, uint32_t* maxs,
                                                              uint32_t* flags) {
  uint32_t mn[4] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu};
  uint32_t mx[4] = {0, 0, 0, 0};
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2], hh = h[i], v = val[i];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !isfinite(v) || !isfinite(hh) || !(hh > 0.0f)) bad = true;
    const float c[4] = {x, y, z, hh};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const uint32_t o = f2ord(c[a]);
      mn[a] = min(mn[a], o);
      mx[a] = max(mx[a], o);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    uint32_t m1 = mn[a], m2 = mx[a];
    for (int o = 32; o >= 1; o >>= 1) {
      m1 = min(m1, (uint32_t)__shfl_xor((int)m1, o, 64));
      m2 = max(m2, (uint32_t)__shfl_xor((int)m2, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      atomicMin(&mins[a], m1);
      atomicMax(&maxs[a], m2);
    }
  }
  if (bad) atomicOr(flags, kFlagBadInput);
}

struct KeyParams {
  double lo[3];
  double c0;
  int bits;  // Morton bits per axis used in the compact sort key
};

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint32_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
  x = (x ^ (x >> 32)) & 0x1fffffull;
  return (uint32_t)x;
}

// sort key: level << (3 bits) | morton(ix, iy, iz); value: input index
__global__ void __launch_bounds__(kThreads) k_keys(const float* xyz, const float* h, int64_t n, KeyParams kp,
                                                   uint64_t* key, uint32_t* idx) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const double qz = kSupport * (double)h[i];
    int l = 0;
    double c = kp.c0;
    while (qz > c) {
      ++l;
      c *= 2.0;
    }
    const double inv = 1.0 / c;
    uint32_t cc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) cc[a] = (uint32_t)floor(((double)xyz[3 * i + a] - kp.lo[a]) * inv);
    const uint64_t m = spread3(cc[0]) | (spread3(cc[1]) << 1) | (spread3(cc[2]) << 2);
    key[i] = ((uint64_t)l << (3 * kp.bits)) | m;
    idx[i] = (uint32_t)i;
  }
}

// ---------------------------------------------------------------- stable LSD radix sort

constexpr int kRadixItems = 16;
constexpr int kRadixTile = kThreads * kRadixItems;

template <class K>
__global__ void __launch_bounds__(kThreads) k_radix_hist(const K* keys, int64_t n, int shift, uint32_t* hist,
                                                         int64_t n_tiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  for (int r = 0; r < kRadixItems; ++r) {
    const int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_u32_to_i64(const uint32_t* a, int64_t* b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

template <class K, bool HAS_VAL>
__global__ void __launch_bounds__(kThreads) k_radix_scatter(const K* keys, const uint32_t* vals, K* keys_out,
                                                            uint32_t* vals_out, int64_t n, int shift,
                                                            const int64_t* offs, int64_t n_tiles) {
  __shared__ int64_t run[256];
  __shared__ uint32_t wcnt[kThreads / 64][256];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  run[tid] = offs[(int64_t)tid * n_tiles + blockIdx.x];
  for (int i = 0; i < kThreads / 64; ++i) wcnt[i][tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kRadixItems; ++r) {
    const int64_t i = base + (int64_t)r * kThreads + tid;
    const bool valid = i < n;
    K k = valid ? keys[i] : K(0);
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((d >> b) & 1u);
      m &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const int rank = __popcll(m & lt);
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (valid) {
      int64_t pos = run[d] + rank;
      for (int ww = 0; ww < w; ++ww) pos += wcnt[ww][d];
      keys_out[pos] = k;
      if (HAS_VAL) vals_out[pos] = vals[i];
    }
    __syncthreads();
    uint32_t tot = 0;
    for (int ww = 0; ww < kThreads / 64; ++ww) {
      tot += wcnt[ww][tid];
      wcnt[ww][tid] = 0;
    }
    run[tid] += tot;
    __syncthreads();
  }
}

// Sorts (keys, vals) by the low `bits` bits of the keys; returns true if the result is in the *_alt buffers.
template <class K>
bool radix_sort(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt, int64_t n, int bits, DevBuf& hist,
                DevBuf& offs, DevBuf& tmp, hipStream_t st) {
  const int64_t tiles = (n + kRadixTile - 1) / kRadixTile;
  hist.ensure(sizeof(uint32_t) * 256 * tiles);
  offs.ensure(sizeof(int64_t) * 256 * tiles * 2);
  int64_t* h64 = offs.as<int64_t>();
  int64_t* o64 = h64 + 256 * tiles;
  bool alt = false;
  for (int shift = 0; shift < bits; shift += 8) {
    K* ki = alt ? keys_alt : keys;
    K* ko = alt ? keys : keys_alt;
    uint32_t* vi = alt ? vals_alt : vals;
    uint32_t* vo = alt ? vals : vals_alt;
    k_radix_hist<K><<<(unsigned)tiles, kThreads, 0, st>>>(ki, n, shift, hist.as<uint32_t>(), tiles);
    k_u32_to_i64<<<256, 256, 0, st>>>(hist.as<uint32_t>(), h64, 256 * tiles);
    device_exclusive_scan_i64(h64, o64, 256 * tiles, tmp, st);
    if (vals)
      k_radix_scatter<K, true><<<(unsigned)tiles, kThreads, 0, st>>>(ki, vi, ko, vo, n, shift, o64, tiles);
    else
      k_radix_scatter<K, false><<<(unsigned)tiles, kThreads, 0, st>>>(ki, nullptr, ko, nullptr, n, shift, o64, tiles);
    hip_check(hipGetLastError(), "radix sort launch");
    alt = !alt;
  }
  return alt;
}

// ---------------------------------------------------------------- permute and cells

__global__ void __launch_bounds__(kThreads) k_permute(const float* xyz, const float* h, const float* v,
                                                      const uint32_t* src, int64_t n, float4* pos4, float* val,
                                                      int32_t* orig) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const uint32_t s = src[i];
    pos4[i] = make_float4(xyz[3 * s], xyz[3 * s + 1], xyz[3 * s + 2], h[s]);
    val[i] = v[s];
    orig[i] = (int32_t)s;
  }
}

__device__ __forceinline__ int64_t cell_linear(const GridDev& g, uint64_t key, int bits, int* level_out) {
  const int l = (int)(key >> (3 * bits));
  const uint64_t m = key & ((uint64_t(1) << (3 * bits)) - 1);
  const uint32_t ix = compact3(m), iy = compact3(m >> 1), iz = compact3(m >> 2);
  const LevelInfo& L = g.lv[l];
  *level_out = l;
  return L.cell_off + (int64_t)ix + (int64_t)L.n[0] * ((int64_t)iy + (int64_t)L.n[1] * (int64_t)iz);
}

__global__ void __launch_bounds__(kThreads) k_cells(const uint64_t* key, int64_t n, GridDev g, int bits,
                                                    uint32_t* cbeg, uint32_t* cend) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const uint64_t k = key[i];
    int l;
    const int64_t c = cell_linear(g, k, bits, &l);
    if (i == 0 || key[i - 1] != k) cbeg[c] = (uint32_t)i;
    if (i + 1 == n || key[i + 1] != k) cend[c] = (uint32_t)(i + 1);
  }
}

// per nonempty cell: sequential float64 sum of |value| w0 / h^3 in index order
__global__ void __launch_bounds__(kThreads) k_cell_sums(const uint64_t* key, const float4* pos4, const float* val,
                                                        int64_t n, GridDev g, int bits, double w0,
                                                        const uint32_t* cend, double* csum) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const uint64_t k = key[i];
    if (i > 0 && key[i - 1] == k) continue;
    int l;
    const int64_t c = cell_linear(g, k, bits, &l);
    const int64_t e = cend[c];
    double s = 0.0;
    for (int64_t j = i; j < e; ++j) {
      const double z = (double)pos4[j].w;
      const double v = fabs((double)val[j]);
      s = s + v * w0 / (z * z * z);
    }
    csum[c] = s;
  }
}

__device__ __forceinline__ double cell_sum_at(const double* csum, const LevelInfo& L, int x, int y, int z) {
  if (x < 0 || y < 0 || z < 0 || x >= L.n[0] || y >= L.n[1] || z >= L.n[2]) return 0.0;
  return csum[L.cell_off + (int64_t)x + (int64_t)L.n[0] * ((int64_t)y + (int64_t)L.n[1] * z)];
}

__global__ void __launch_bounds__(kThreads) k_nbhd_max(const double* csum, GridDev g, int level,
                                                       unsigned long long* lmax) {
  const LevelInfo& L = g.lv[level];
  const int64_t ex = L.n[0] + 2, ey = L.n[1] + 2, ez = L.n[2] + 2;
  const int64_t total = ex * ey * ez;
  double best = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total; i += (int64_t)gridDim.x * kThreads) {
    const int x = (int)(i % ex) - 1, y = (int)((i / ex) % ey) - 1, z = (int)(i / (ex * ey)) - 1;
    double acc = 0.0;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) acc = acc + cell_sum_at(csum, L, x + dx, y + dy, z + dz);
    best = fmax(best, acc);
  }
  unsigned long long b = (unsigned long long)__double_as_longlong(best);
  for (int o = 32; o >= 1; o >>= 1) {
    unsigned long long nb = __shfl_xor(b, o, 64);
    b = b > nb ? b : nb;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(lmax, b);
}

__global__ void __launch_bounds__(kThreads) k_repr_keys(const float4* pos4, const float* val, int64_t n,
                                                        uint32_t* hkey, uint64_t* pkey) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const float hz = pos4[i].w;
    hkey[i] = __float_as_uint(hz);  // h > 0: bit patterns order like the values
    const double z = (double)hz;
    const double phi = fabs((double)val[i]) / (z * z * z);
    pkey[i] = (uint64_t)__double_as_longlong(phi);  // >= 0
  }
}

__global__ void k_level_of(const uint64_t* key, int64_t n, int bits, int32_t* level, uint64_t* morton) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = key[i];
    if (level) level[i] = (int32_t)(k >> (3 * bits));
    if (morton) morton[i] = k & ((uint64_t(1) << (3 * bits)) - 1);
  }
}

double pow2_at_least(double x) {
  int e;
  const double m = std::frexp(x, &e);
  return m == 0.5 ? std::ldexp(1.0, e - 1) : std::ldexp(1.0, e);
}

unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 8192)); }

}  // namespace

bool device_sort_u64(uint64_t* keys, uint64_t* alt, int64_t n, int bits, DevBuf& hist, DevBuf& offs, DevBuf& tmp,
                     hipStream_t st) {
  return radix_sort<uint64_t>(keys, nullptr, alt, nullptr, n, bits, hist, offs, tmp, st);
}

void build_index_device(Index& ix, const float* xyz, const float* h, const float* value, hipStream_t st) {
  const int64_t n = ix.n;
  DevBuf small;
  small.ensure(64);
  uint32_t init[12];
  for (int a = 0; a < 4; ++a) {
    init[a] = 0xffffffffu;
    init[4 + a] = 0u;
  }
  init[8] = 0;
  hip_check(hipMemcpyAsync(small.p, init, sizeof(uint32_t) * 9, hipMemcpyHostToDevice, st), "copy");
  uint32_t* mins = small.as<uint32_t>();
  k_validate_bounds<<<grid_for(n), kThreads, 0, st>>>(xyz, h, value, n, mins, mins + 4, mins + 8);
  hip_check(hipGetLastError(), "validate launch");
  uint32_t got[9];
  hip_check(hipMemcpyAsync(got, small.p, sizeof(uint32_t) * 9, hipMemcpyDeviceToHost, st), "copy");
  hip_check(hipStreamSynchronize(st), "sync");
  if (got[8] & kFlagBadInput) throw Error(SPH_HOA_E_INVALID_ARG, "particle data contains NaN/inf or h <= 0");
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = (double)ord2f(got[a]);
    hi[a] = (double)ord2f(got[4 + a]);
  }
  const double hmin = (double)ord2f(got[3]), hmax = (double)ord2f(got[7]);
  // levels
  double c0 = pow2_at_least(kSupport * hmin);
  auto dims = [&](double c, int64_t* d) {
    for (int a = 0; a < 3; ++a) d[a] = (int64_t)std::floor((hi[a] - lo[a]) * (1.0 / c)) + 1;
  };
  for (;;) {
    int64_t d[3];
    dims(c0, d);
    if ((double)d[0] * (double)d[1] * (double)d[2] > (double)kMaxLevel0Cells || d[0] > kMaxAxisCells ||
        d[1] > kMaxAxisCells || d[2] > kMaxAxisCells)
      c0 *= 2.0;
    else
      break;
  }
  int n_levels = 1;
  {
    double c = c0;
    while (kSupport * hmax > c) {
      c *= 2.0;
      ++n_levels;
    }
  }
  if (n_levels > kMaxLevels) throw Error(SPH_HOA_E_UNSUPPORTED, "smoothing lengths span more than 2^31");
  GridDev g{};
  int64_t cell_total = 0;
  int64_t maxdim = 1;
  for (int a = 0; a < 3; ++a) g.lo[a] = lo[a];
  g.n_levels = n_levels;
  for (int l = 0; l < n_levels; ++l) {
    const double c = std::ldexp(c0, l);
    int64_t d[3];
    dims(c, d);
    g.lv[l].c = c;
    g.lv[l].inv_c = 1.0 / c;
    for (int a = 0; a < 3; ++a) {
      g.lv[l].n[a] = (int)d[a];
      maxdim = std::max(maxdim, d[a]);
    }
    g.lv[l].cell_off = cell_total;
    cell_total += d[0] * d[1] * d[2];
  }
  int bits = 1;
  while ((int64_t(1) << bits) < maxdim) ++bits;
  int lbits = 1;
  while ((1 << lbits) < n_levels) ++lbits;
  KeyParams kp;
  for (int a = 0; a < 3; ++a) kp.lo[a] = lo[a];
  kp.c0 = c0;
  kp.bits = bits;
  // keys and stable sort
  DevBuf key_a, key_b, val_a, val_b, hist, offs, tmp;
  key_a.ensure(8 * n);
  key_b.ensure(8 * n);
  val_a.ensure(4 * n);
  val_b.ensure(4 * n);
  k_keys<<<grid_for(n), kThreads, 0, st>>>(xyz, h, n, kp, key_a.as<uint64_t>(), val_a.as<uint32_t>());
  hip_check(hipGetLastError(), "keys launch");
  const bool alt = radix_sort<uint64_t>(key_a.as<uint64_t>(), val_a.as<uint32_t>(), key_b.as<uint64_t>(),
                                        val_b.as<uint32_t>(), n, 3 * bits + lbits, hist, offs, tmp, st);
  uint64_t* skey = alt ? key_b.as<uint64_t>() : key_a.as<uint64_t>();
  uint32_t* sval = alt ? val_b.as<uint32_t>() : val_a.as<uint32_t>();
  ix.pos4.ensure(sizeof(float4) * n);
  ix.val.ensure(sizeof(float) * n);
  ix.orig.ensure(sizeof(int32_t) * n);
  ix.morton.ensure(sizeof(uint64_t) * n);
  k_permute<<<grid_for(n), kThreads, 0, st>>>(xyz, h, value, sval, n, ix.pos4.as<float4>(), ix.val.as<float>(),
                                              ix.orig.as<int32_t>());
  hip_check(hipMemcpyAsync(ix.morton.p, skey, 8 * n, hipMemcpyDeviceToDevice, st), "copy");
  ix.cell_begin.ensure(sizeof(uint32_t) * cell_total);
  ix.cell_end.ensure(sizeof(uint32_t) * cell_total);
  hip_check(hipMemsetAsync(ix.cell_begin.p, 0, sizeof(uint32_t) * cell_total, st), "memset");
  hip_check(hipMemsetAsync(ix.cell_end.p, 0, sizeof(uint32_t) * cell_total, st), "memset");
  k_cells<<<grid_for(n), kThreads, 0, st>>>(skey, n, g, bits, ix.cell_begin.as<uint32_t>(), ix.cell_end.as<uint32_t>());
  hip_check(hipGetLastError(), "cells launch");
  // per-level particle counts (host, from the sorted keys' level boundaries)
  {
    DevBuf lv;
    lv.ensure(sizeof(int32_t) * n);
    k_level_of<<<grid_for(n), kThreads, 0, st>>>(skey, n, bits, lv.as<int32_t>(), nullptr);
    std::vector<int32_t> levels(n);
    hip_check(hipMemcpyAsync(levels.data(), lv.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st), "copy");
    hip_check(hipStreamSynchronize(st), "sync");
    for (int l = 0; l < n_levels; ++l) g.lv[l].n_particles = 0;
    for (int64_t i = 0; i < n; ++i) g.lv[levels[i]].n_particles++;
  }
  // a_max (unless given)
  if (!(ix.a_max > 0.0)) {
    DevBuf csum, lmax;
    csum.ensure(sizeof(double) * cell_total);
    lmax.ensure(sizeof(unsigned long long) * kMaxLevels);
    hip_check(hipMemsetAsync(csum.p, 0, sizeof(double) * cell_total, st), "memset");
    hip_check(hipMemsetAsync(lmax.p, 0, sizeof(unsigned long long) * kMaxLevels, st), "memset");
    k_cell_sums<<<grid_for(n), kThreads, 0, st>>>(skey, ix.pos4.as<float4>(), ix.val.as<float>(), n, g, bits,
                                                  kernel_w0(ix.kernel), ix.cell_end.as<uint32_t>(), csum.as<double>());
    for (int l = 0; l < n_levels; ++l) {
      const int64_t tot = (int64_t)(g.lv[l].n[0] + 2) * (g.lv[l].n[1] + 2) * (g.lv[l].n[2] + 2);
      k_nbhd_max<<<grid_for(tot), kThreads, 0, st>>>(csum.as<double>(), g, l, lmax.as<unsigned long long>() + l);
    }
    hip_check(hipGetLastError(), "a_max launch");
    unsigned long long lm[kMaxLevels];
    hip_check(hipMemcpyAsync(lm, lmax.p, sizeof(lm), hipMemcpyDeviceToHost, st), "copy");
    hip_check(hipStreamSynchronize(st), "sync");
    double total = 0.0;
    for (int l = 0; l < n_levels; ++l) {
      double v;
      memcpy(&v, &lm[l], 8);
      total = total + v;
    }
    ix.a_max = kAmaxMargin * total;
  }
  // representative attributes (lower medians), unless given
  if (!(ix.h_repr > 0.0) || !(ix.phi_repr > 0.0)) {
    DevBuf hk, hk2, pk, pk2;
    hk.ensure(4 * n);
    hk2.ensure(4 * n);
    pk.ensure(8 * n);
    pk2.ensure(8 * n);
    k_repr_keys<<<grid_for(n), kThreads, 0, st>>>(ix.pos4.as<float4>(), ix.val.as<float>(), n, hk.as<uint32_t>(),
                                                  pk.as<uint64_t>());
    const bool a1 = radix_sort<uint32_t>(hk.as<uint32_t>(), nullptr, hk2.as<uint32_t>(), nullptr, n, 32, hist, offs,
                                         tmp, st);
    const bool a2 = radix_sort<uint64_t>(pk.as<uint64_t>(), nullptr, pk2.as<uint64_t>(), nullptr, n, 64, hist, offs,
                                         tmp, st);
    const int64_t mid = (n - 1) / 2;
    uint32_t hb;
    uint64_t pb;
    hip_check(hipMemcpyAsync(&hb, (a1 ? hk2.as<uint32_t>() : hk.as<uint32_t>()) + mid, 4, hipMemcpyDeviceToHost, st),
              "copy");
    hip_check(hipMemcpyAsync(&pb, (a2 ? pk2.as<uint64_t>() : pk.as<uint64_t>()) + mid, 8, hipMemcpyDeviceToHost, st),
              "copy");
    hip_check(hipStreamSynchronize(st), "sync");
    float hf;
    double pd;
    memcpy(&hf, &hb, 4);
    memcpy(&pd, &pb, 8);
    if (!(ix.h_repr > 0.0)) ix.h_repr = (double)hf;
    if (!(ix.phi_repr > 0.0)) ix.phi_repr = pd;
  }
  hip_check(hipStreamSynchronize(st), "sync");
  ix.grid = g;
  ix.cell0 = c0;
  ix.grid_bits = bits;
}

// Clears *diff if every particle record (position and smoothing length, input index) is equal in
// both indices; grid-stride, any grid.
__global__ void __launch_bounds__(256) k_same_particles(const float4* a, const float4* b, const int32_t* oa,
                                                        const int32_t* ob, int64_t n, unsigned int* diff) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float4 p = a[i], q = b[i];
    const bool same = __float_as_uint(p.x) == __float_as_uint(q.x) && __float_as_uint(p.y) == __float_as_uint(q.y) &&
                      __float_as_uint(p.z) == __float_as_uint(q.z) && __float_as_uint(p.w) == __float_as_uint(q.w) &&
                      oa[i] == ob[i];
    if (!same) atomicOr(diff, 1u);
  }
}

bool same_particles(const Index& a, const Index& b, hipStream_t st) {
  if (a.n != b.n) return false;
  if (a.n == 0) return true;
  DevBuf d;
  d.ensure(sizeof(unsigned int));
  unsigned int* diff = d.as<unsigned int>();
  hip_check(hipMemsetAsync(diff, 0, sizeof(unsigned int), st), "memset");
  k_same_particles<<<grid_for(a.n), kThreads, 0, st>>>(a.pos4.as<float4>(), b.pos4.as<float4>(), a.orig.as<int32_t>(),
                                                       b.orig.as<int32_t>(), a.n, diff);
  hip_check(hipGetLastError(), "compare launch");
  unsigned int h = 1;
  hip_check(hipMemcpyAsync(&h, diff, sizeof(h), hipMemcpyDeviceToHost, st), "copy");
  hip_check(hipStreamSynchronize(st), "sync");
  return h == 0;
}

void get_grid_device(Index& ix, uint64_t* morton, int32_t* level, int32_t* order, hipStream_t st) {
  const int64_t n = ix.n;
  k_level_of<<<grid_for(n), kThreads, 0, st>>>(ix.morton.as<uint64_t>(), n, ix.grid_bits, level, morton);
  if (order) hip_check(hipMemcpyAsync(order, ix.orig.p, 4 * n, hipMemcpyDeviceToDevice, st), "copy");
  hip_check(hipGetLastError(), "grid launch");
  hip_check(hipStreamSynchronize(st), "sync");
}

}  // namespace sph
