// Per-frame path: rays, hit gathering, and the per-ray field kernel.
//
// Sec. 2 describes three passes: (1) approximate every particle on all rays
// it affects, (2) sort each ray's knots by position, (3) accumulate them,
// classify and composite.  Here pass 1 is split into a hit-gathering kernel
// (one wave per ray walks the multi-level grid and tests candidates with the
// exact float64 predicate) and the knot generation inside the per-ray
// kernel, which then sorts, accumulates (Eq. accumulation-rule, exact in
// wrap-around 64-bit integers), merges and either writes the merged pieces or
// composites them - all for one ray per work-group, in LDS.
#include <hip/hip_runtime.h>

#include <memory>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "device.h"
#include "impl.h"

namespace sph {

namespace {

// ============================================================== rays

struct CamDev {
  double eye[3], f[3], r[3], u[3];
  double g, aspect, half;  // tan(fov/2), W/H, ortho half extent
  int W, H, ortho;
  float t_min, t_max;
};

// Ray of pixel p (row-major, row 0 at the top) through the pixel centre.
__device__ __forceinline__ void camera_ray(const CamDev& c, int64_t p, double* o, double* v) {
  const double col = (double)(p % c.W), row = (double)(p / c.W);
  const double a = (2.0 * col + 1.0) / (double)c.W - 1.0;
  const double b = 1.0 - (2.0 * row + 1.0) / (double)c.H;
  if (c.ortho) {
    const double sa = a * c.half * c.aspect, sb = b * c.half;
    for (int k = 0; k < 3; ++k) {
      o[k] = c.eye[k] + sa * c.r[k] + sb * c.u[k];
      v[k] = c.f[k];
    }
  } else {
    const double sa = a * c.g * c.aspect, sb = b * c.g;
    const double dx = c.f[0] + sa * c.r[0] + sb * c.u[0];
    const double dy = c.f[1] + sa * c.r[1] + sb * c.u[1];
    const double dz = c.f[2] + sa * c.r[2] + sb * c.u[2];
    const double nrm = sqrt(dx * dx + dy * dy + dz * dz);
    v[0] = dx / nrm;
    v[1] = dy / nrm;
    v[2] = dz / nrm;
    for (int k = 0; k < 3; ++k) o[k] = c.eye[k];
  }
}

// Rays of one or more cameras, concatenated in camera order (offs: first ray of each camera, n_cams + 1
// entries), with each ray's own segment [t_min, t_max] in tr.
__global__ void k_camera_rays_batch(const CamDev* cams, const int64_t* offs, int n_cams, int64_t n, double* o,
                                    double* v, float* tr) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = n_cams - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (offs[mid] <= p) lo = mid;
      else hi = mid - 1;
    }
    const CamDev& c = cams[lo];
    camera_ray(c, p - offs[lo], o + 3 * p, v + 3 * p);
    tr[2 * p] = c.t_min;
    tr[2 * p + 1] = c.t_max;
  }
}

__global__ void k_low32(const uint64_t* keys, int64_t n, uint32_t* out) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
    out[p] = (uint32_t)keys[p];
}

// Longest first (rays by hits, tiles by candidates): key = (2^32 - 1 - count) << 32 | index,
// sorted ascending.
__global__ void k_order_keys(const int64_t* count, int64_t n, uint64_t* keys) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t c = (uint64_t)min(count[p], (int64_t)0xffffffff);
    keys[p] = ((0xffffffffull - c) << 32) | (uint64_t)p;
  }
}

__global__ void k_widen_rays(const float* of, const float* vf, int64_t n, double* o, double* v, uint32_t* flags) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    bool bad = false;
    for (int k = 0; k < 3; ++k) {
      const float a = of[3 * p + k], b = vf[3 * p + k];
      if (!isfinite(a) || !isfinite(b)) bad = true;
      o[3 * p + k] = (double)a;
      v[3 * p + k] = (double)b;
      s += (double)b * (double)b;
    }
    if (bad || !(fabs(s - 1.0) <= 1e-5)) atomicOr(flags, kFlagBadInput);
  }
}

// ============================================================== hit gathering

constexpr int kGatherThreads = 256;  // four waves, one ray each

struct GatherArgs {
  const double* o;
  const double* v;
  int64_t n_rays;
  double t_min, t_max;
  const float* tr;      // optional per-ray [t_min, t_max] (batches); else the scalars above
  const float4* pos4;
  const uint32_t* cbeg;
  const uint32_t* cend;
  GridDev g;
  int64_t* count;       // count pass: hits per ray
  const int64_t* off;   // fill pass: offsets
  uint32_t* hits;       // fill pass: permuted particle indices
  uint32_t* slots;      // count pass, optional: ray r's first n_slots hits at [r * n_slots, ...)
  int64_t n_slots;
  unsigned long long* max_hits;
  uint32_t* flags;
};

// Exact contribution test (same float64 operation order as the oracle).
__device__ __forceinline__ bool pair_hit(const double o[3], const double v[3], float4 p, double t_min, double t_max) {
  const double dxx = (double)p.x - o[0], dxy = (double)p.y - o[1], dxz = (double)p.z - o[2];
  const double cx = dxy * v[2] - dxz * v[1];
  const double cy = dxz * v[0] - dxx * v[2];
  const double cz = dxx * v[1] - dxy * v[0];
  const double z = (double)p.w;
  const double lam2 = (cx * cx + cy * cy + cz * cz) / (z * z);
  if (!(lam2 < kSupport * kSupport)) return false;
  const double tchi = dxx * v[0] + dxy * v[1] + dxz * v[2];
  // s z >= 0 and rounding is monotone, so fl(tchi + s z) >= tchi and fl(tchi - s z) <= tchi: a
  // centre strictly inside (t_min, t_max) passes both end tests whatever s is, and the square
  // root is only needed for the others (same decisions as evaluating both tests).
  if (tchi > t_min && tchi < t_max) return true;
  const double s = sqrt(kSupport * kSupport - lam2);
  const double sz = s * z;
  return (tchi + sz > t_min) && (tchi - sz < t_max);
}

template <bool FILL>
__global__ void __launch_bounds__(kGatherThreads) k_gather(GatherArgs A) {
  __shared__ int64_t s_excl[kGatherThreads];
  __shared__ uint32_t s_beg[kGatherThreads];
  __shared__ int32_t s_cfirst[kGatherThreads], s_cb0[kGatherThreads], s_ce0[kGatherThreads], s_cne[kGatherThreads];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * (kGatherThreads / 64) + w;
  if (r >= A.n_rays) return;  // whole wave leaves together
  double o[3], v[3];
  for (int k = 0; k < 3; ++k) {
    o[k] = A.o[3 * r + k];
    v[k] = A.v[3 * r + k];
  }
  const double t_min = A.tr ? (double)A.tr[2 * r] : A.t_min, t_max = A.tr ? (double)A.tr[2 * r + 1] : A.t_max;
  int64_t* ex = s_excl + w * 64;
  uint32_t* bg = s_beg + w * 64;
  int32_t *sx = s_cfirst + w * 64, *sb = s_cb0 + w * 64, *se = s_ce0 + w * 64, *sn = s_cne + w * 64;
  int64_t found = 0;
  const int64_t out0 = FILL ? A.off[r] : 0;
  // dominant axis
  int ax = 0;
  if (fabs(v[1]) > fabs(v[ax])) ax = 1;
  if (fabs(v[2]) > fabs(v[ax])) ax = 2;
  const int bx = (ax + 1) % 3, ex_ax = (ax + 2) % 3;
  for (int l = 0; l < A.g.n_levels; ++l) {
    const LevelInfo& L = A.g.lv[l];
    if (L.n_particles == 0) continue;
    const double c = L.c, ic = L.inv_c, eps = c * 1e-7;
    // clip the segment to the box in which it can reach this level's particles
    double ta = t_min, tb = t_max;
    bool empty = false;
    for (int a = 0; a < 3; ++a) {
      const double bmin = A.g.lo[a] - c - eps, bmax = A.g.lo[a] + (double)(L.n[a] + 1) * c + eps;
      if (v[a] == 0.0) {
        if (o[a] < bmin || o[a] > bmax) empty = true;
      } else {
        double t1 = (bmin - o[a]) / v[a], t2 = (bmax - o[a]) / v[a];
        if (t1 > t2) {
          const double tt = t1;
          t1 = t2;
          t2 = tt;
        }
        ta = fmax(ta, t1);
        tb = fmin(tb, t2);
      }
    }
    if (empty || !(ta <= tb)) continue;
    const double a0 = o[ax] + ta * v[ax], a1 = o[ax] + tb * v[ax];
    int64_t s_lo = (int64_t)floor((fmin(a0, a1) - c - eps - A.g.lo[ax]) * ic);
    int64_t s_hi = (int64_t)floor((fmax(a0, a1) + c + eps - A.g.lo[ax]) * ic);
    s_lo = max(s_lo, (int64_t)0);
    s_hi = min(s_hi, (int64_t)L.n[ax] - 1);
    if (s_hi < s_lo) continue;
    // The slabs of this level 64 at a time, one lane per slab: each lane finds its slab's window
    // of cells in the two other axes (the segment's crossing of the slab and its two neighbours,
    // widened by one cell; at most 7 x 7), then the chunk's cells are visited 64 at a time in
    // (slab, b, e) order, so every lane of a batch holds a real cell.
    for (int64_t s_base = s_lo; s_base <= s_hi; s_base += 64) {
      const int64_t s = s_base + lane;
      int nb = 0, ne = 0;
      int64_t cb0 = 0, ce0 = 0;
      if (s <= s_hi) {
        double t1 = (A.g.lo[ax] + (double)(s - 1) * c - eps - o[ax]) / v[ax];
        double t2 = (A.g.lo[ax] + (double)(s + 2) * c + eps - o[ax]) / v[ax];
        if (t1 > t2) {
          const double tt = t1;
          t1 = t2;
          t2 = tt;
        }
        t1 = fmax(t1, ta);
        t2 = fmin(t2, tb);
        if (t1 <= t2) {
          const double b1 = o[bx] + t1 * v[bx], b2 = o[bx] + t2 * v[bx];
          const double e1 = o[ex_ax] + t1 * v[ex_ax], e2 = o[ex_ax] + t2 * v[ex_ax];
          int64_t cb_lo = (int64_t)floor((fmin(b1, b2) - c - eps - A.g.lo[bx]) * ic);
          int64_t cb_hi = (int64_t)floor((fmax(b1, b2) + c + eps - A.g.lo[bx]) * ic);
          int64_t ce_lo = (int64_t)floor((fmin(e1, e2) - c - eps - A.g.lo[ex_ax]) * ic);
          int64_t ce_hi = (int64_t)floor((fmax(e1, e2) + c + eps - A.g.lo[ex_ax]) * ic);
          if (cb_hi - cb_lo > 6 || ce_hi - ce_lo > 6) atomicOr(A.flags, kFlagWindow);
          cb_lo = max(cb_lo, (int64_t)0);
          ce_lo = max(ce_lo, (int64_t)0);
          cb_hi = min(min(cb_hi, (int64_t)L.n[bx] - 1), cb_lo + 6);
          ce_hi = min(min(ce_hi, (int64_t)L.n[ex_ax] - 1), ce_lo + 6);
          if (cb_hi >= cb_lo && ce_hi >= ce_lo) {
            nb = (int)(cb_hi - cb_lo + 1);
            ne = (int)(ce_hi - ce_lo + 1);
            cb0 = cb_lo;
            ce0 = ce_lo;
          }
        }
      }
      const int ncell = nb * ne;
      const int cincl = (int)wave_incl_scan((int64_t)ncell);
      const int ctot = __shfl(cincl, 63, 64);
      sx[lane] = cincl - ncell;
      sb[lane] = (int32_t)cb0;
      se[lane] = (int32_t)ce0;
      sn[lane] = ne;
      __builtin_amdgcn_wave_barrier();
      for (int cbase = 0; cbase < ctot; cbase += 64) {
        const int ci0 = cbase + lane;
        int64_t cnt = 0;
        uint32_t cb = 0;
        if (ci0 < ctot) {
          // owner lane: last lane whose first cell is <= ci0 (lanes without cells share the next
          // lane's first cell, so the search ends on a lane with cells)
          int lo = 0, hi = 63;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sx[mid] <= ci0) lo = mid;
            else hi = mid - 1;
          }
          const int li = ci0 - sx[lo], nel = sn[lo];
          int64_t cc[3];
          cc[ax] = s_base + lo;
          cc[bx] = (int64_t)sb[lo] + li / nel;
          cc[ex_ax] = (int64_t)se[lo] + li % nel;
          const int64_t cell = L.cell_off + cc[0] + (int64_t)L.n[0] * (cc[1] + (int64_t)L.n[1] * cc[2]);
          cb = A.cbeg[cell];
          cnt = (int64_t)A.cend[cell] - (int64_t)cb;
        }
        const int64_t incl = wave_incl_scan(cnt);
        const int64_t tot = __shfl(incl, 63, 64);
        ex[lane] = incl - cnt;
        bg[lane] = cb;
        __builtin_amdgcn_wave_barrier();
        for (int64_t k = 0; k < tot; k += 64) {
          const int64_t ci = k + lane;
          bool hit = false;
          uint32_t j = 0;
          if (ci < tot) {
            // owner lane: last lane with ex <= ci
            int lo = 0, hi = 63;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (ex[mid] <= ci) lo = mid;
              else hi = mid - 1;
            }
            j = bg[lo] + (uint32_t)(ci - ex[lo]);
            hit = pair_hit(o, v, A.pos4[j], t_min, t_max);
          }
          const uint64_t m = __ballot(hit);
          if (hit) {
            const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
            const int64_t pos = found + __popcll(m & lt);
            if (FILL) A.hits[out0 + pos] = j;
            else if (A.slots && pos < A.n_slots) A.slots[r * A.n_slots + pos] = j;
          }
          found += __popcll(m);
        }
        __builtin_amdgcn_wave_barrier();
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (!FILL && lane == 0) {
    A.count[r] = found;
    atomicMax(A.max_hits, (unsigned long long)found);
  }
}

// ============================================================== camera rays: screen-tile binning
//
// For camera rays the relevant rays of a particle (Sec. 2, first pass) are the pixels inside the
// projection of its support sphere.  Each particle is binned into the 8 x 8-pixel tiles its
// projection's bounding box covers (a conservative box with a one-pixel margin; spheres that
// reach the eye plane cover every tile); the exact float64 test then decides per (pixel ray,
// candidate).  Replaces the grid walk for rendering: every tile's rays share one candidate list.

constexpr int kTile = 8;

struct BinArgs {
  const float4* pos4;
  int64_t n;
  const CamDev* cams;       // [n_cams]
  const int64_t* tile_base; // [n_cams + 1] first tile of each camera in the concatenated tile index
  int n_cams;
  unsigned int* tile_count;
  const int64_t* tile_off;
  unsigned int* tile_cursor;
  uint32_t* items;
};

// pixel range [c0, c1] x [r0, r1] of camera c covered by the projection of the particle's support sphere
__device__ bool particle_pixels(const CamDev& c, float4 p, int* c0, int* c1, int* r0, int* r1) {
  const double t_min = (double)c.t_min, t_max = (double)c.t_max;
  const double dx = (double)p.x - c.eye[0], dy = (double)p.y - c.eye[1], dz = (double)p.z - c.eye[2];
  const double z = dx * c.f[0] + dy * c.f[1] + dz * c.f[2];
  const double x = dx * c.r[0] + dy * c.r[1] + dz * c.r[2];
  const double y = dx * c.u[0] + dy * c.u[1] + dz * c.u[2];
  const double R = kSupport * (double)p.w * (1.0 + 1e-6) + 1e-12;
  double a0, a1, b0, b1;
  if (c.ortho) {
    if (z + R < t_min || z - R > t_max) return false;
    a0 = (x - R) / (c.half * c.aspect);
    a1 = (x + R) / (c.half * c.aspect);
    b0 = (y - R) / c.half;
    b1 = (y + R) / c.half;
  } else {
    const double dist = sqrt(dx * dx + dy * dy + dz * dz);
    if (dist - R >= t_max || dist + R <= t_min) return false;
    if (z <= R * 1.0001) {
      a0 = b0 = -1e30;
      a1 = b1 = 1e30;
    } else {
      // In the (x, z) plane the sphere is seen at angle theta (tan theta = x / z) with half-width
      // alpha (sin alpha = R / sqrt(x^2 + z^2)); the screen bounds are tan(theta -+ alpha), by the
      // tangent addition formula with tan alpha = R / sqrt(x^2 + z^2 - R^2).  A bound is unbounded
      // when theta -+ alpha leaves (-pi/2, pi/2), i.e. when cos(theta -+ alpha), whose sign is that
      // of 1 +- tan theta tan alpha, is not positive.  Same for (y, z).
      const double tx = x / z, ty = y / z;
      const double sx = R / sqrt(x * x + z * z - R * R), sy = R / sqrt(y * y + z * z - R * R);
      const double dx0 = 1.0 + tx * sx, dx1 = 1.0 - tx * sx, dy0 = 1.0 + ty * sy, dy1 = 1.0 - ty * sy;
      a0 = (dx0 <= 0.0) ? -1e30 : (tx - sx) / dx0 / (c.g * c.aspect);
      a1 = (dx1 <= 0.0) ? 1e30 : (tx + sx) / dx1 / (c.g * c.aspect);
      b0 = (dy0 <= 0.0) ? -1e30 : (ty - sy) / dy0 / c.g;
      b1 = (dy1 <= 0.0) ? 1e30 : (ty + sy) / dy1 / c.g;
    }
  }
  // a = (2 col + 1) / W - 1  and  b = 1 - (2 row + 1) / H
  const double W = (double)c.W, H = (double)c.H;
  const double fc0 = fmax(-2.0, fmin(W + 2.0, ((a0 + 1.0) * W - 1.0) * 0.5));
  const double fc1 = fmax(-2.0, fmin(W + 2.0, ((a1 + 1.0) * W - 1.0) * 0.5));
  const double fr0 = fmax(-2.0, fmin(H + 2.0, ((1.0 - b1) * H - 1.0) * 0.5));
  const double fr1 = fmax(-2.0, fmin(H + 2.0, ((1.0 - b0) * H - 1.0) * 0.5));
  *c0 = max(0, (int)floor(fc0) - 1);
  *c1 = min(c.W - 1, (int)ceil(fc1) + 1);
  *r0 = max(0, (int)floor(fr0) - 1);
  *r1 = min(c.H - 1, (int)ceil(fr1) + 1);
  return *c0 <= *c1 && *r0 <= *r1;
}

// (camera, particle) pairs, camera-major so that consecutive threads read consecutive particles.
// A particle can cover anything from one tile to hundreds (zoomed views), so each wave first
// projects its 64 pairs and then walks the union of their (pair, tile) items 64 at a time: every
// lane takes one item (its owner pair found by binary search in the wave's prefix sums).
template <bool FILL>
__global__ void __launch_bounds__(256) k_bin(BinArgs B) {
  __shared__ int64_t s_ex[256];
  __shared__ int64_t s_tb[256];
  __shared__ int32_t s_tx0[256], s_w[256], s_ty0[256], s_tilesx[256];
  __shared__ uint32_t s_j[256];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int64_t* ex = s_ex + wv * 64;
  int64_t* tb = s_tb + wv * 64;
  int32_t *tx0 = s_tx0 + wv * 64, *wd = s_w + wv * 64, *ty0 = s_ty0 + wv * 64, *tsx = s_tilesx + wv * 64;
  uint32_t* jj = s_j + wv * 64;
  const int64_t total = B.n * (int64_t)B.n_cams;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = base + threadIdx.x;
    int64_t ntiles = 0;
    if (i < total) {
      const int cam = (int)(i / B.n);
      const int64_t j = i - (int64_t)cam * B.n;
      const CamDev& c = B.cams[cam];
      int c0, c1, r0, r1;
      if (particle_pixels(c, B.pos4[j], &c0, &c1, &r0, &r1)) {
        const int x0 = c0 / kTile, x1 = c1 / kTile, y0 = r0 / kTile, y1 = r1 / kTile;
        ntiles = (int64_t)(x1 - x0 + 1) * (y1 - y0 + 1);
        tx0[lane] = x0;
        wd[lane] = x1 - x0 + 1;
        ty0[lane] = y0;
        tsx[lane] = (c.W + kTile - 1) / kTile;
        tb[lane] = B.tile_base[cam];
        jj[lane] = (uint32_t)j;
      }
    }
    const int64_t incl = wave_incl_scan(ntiles);
    const int64_t tot = __shfl(incl, 63, 64);
    ex[lane] = incl - ntiles;
    __builtin_amdgcn_wave_barrier();
    for (int64_t k = 0; k < tot; k += 64) {
      const int64_t q = k + lane;
      if (q < tot) {
        // owner: the last lane whose first item is <= q (lanes without items share the next
        // lane's start, so the search never stops on one of them)
        int lo = 0, hi = 63;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (ex[mid] <= q) lo = mid;
          else hi = mid - 1;
        }
        const int local = (int)(q - ex[lo]);  // < tiles of one image < 2^25
        const int64_t t = tb[lo] + (int64_t)(ty0[lo] + local / wd[lo]) * tsx[lo] + tx0[lo] + local % wd[lo];
        if (FILL) {
          const unsigned int kk = atomicAdd(&B.tile_cursor[t], 1u);
          B.items[B.tile_off[t] + kk] = jj[lo];
        } else {
          atomicAdd(&B.tile_count[t], 1u);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ void k_u32_to_i64_n(const unsigned int* a, int64_t* b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

struct TileHitArgs {
  const double* o;
  const double* v;
  const CamDev* cams;
  const int64_t* tile_base;  // [n_cams + 1]
  const int64_t* ray_base;   // [n_cams + 1] first ray of each camera
  int n_cams;
  const float4* pos4;
  const int64_t* tile_off;
  const uint32_t* items;
  unsigned long long* masks;  // [items]: pixels of the tile each candidate hits (bit = lane)
  const uint32_t* order;      // tiles in order of decreasing candidate count (the heavy ones start first)
  int64_t* count;
  const int64_t* off;
  uint32_t* hits;
  unsigned long long* max_hits;
};

// One wave per tile, one lane per pixel ray; candidates staged through LDS 64 at a time.  The
// counting pass tests every (candidate, pixel) pair and keeps, per candidate, the wave's 64-bit
// mask of the pixels it hits; the filling pass only reads the masks back, so the float64 tests
// run once.  Hits are written in candidate order in both layouts.
template <bool FILL>
__global__ void __launch_bounds__(64) k_tile_hits(TileHitArgs T) {
  __shared__ float4 cp[64];
  __shared__ uint32_t cj[64];
  __shared__ unsigned long long cm[64];
  const int64_t tile = T.order[blockIdx.x];
  const int lane = threadIdx.x;
  int lo = 0, hi = T.n_cams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (T.tile_base[mid] <= tile) lo = mid;
    else hi = mid - 1;
  }
  const CamDev& c = T.cams[lo];
  const double t_min = (double)c.t_min, t_max = (double)c.t_max;
  const int64_t lt = tile - T.tile_base[lo];
  const int tiles_x = (c.W + kTile - 1) / kTile;
  const int tx = (int)(lt % tiles_x), ty = (int)(lt / tiles_x);
  const int col = tx * kTile + (lane % kTile), row = ty * kTile + (lane / kTile);
  const bool valid = col < c.W && row < c.H;
  const int64_t r = valid ? T.ray_base[lo] + (int64_t)row * c.W + col : 0;
  double o[3] = {0, 0, 0}, v[3] = {0, 0, 1};
  if (!FILL && valid)
    for (int k = 0; k < 3; ++k) {
      o[k] = T.o[3 * r + k];
      v[k] = T.v[3 * r + k];
    }
  const int64_t b = T.tile_off[tile], e = T.tile_off[tile + 1];
  int64_t cnt = 0;
  const int64_t out0 = (FILL && valid) ? T.off[r] : 0;
  for (int64_t base = b; base < e; base += 64) {
    const int64_t k = base + lane;
    if (k < e) {
      const uint32_t j = T.items[k];
      cj[lane] = j;
      if (FILL) cm[lane] = T.masks[k];
      else cp[lane] = T.pos4[j];
    }
    __syncthreads();
    const int m = (int)min((int64_t)64, e - base);
    if (FILL) {
      if (valid)
        for (int q = 0; q < m; ++q)
          if ((cm[q] >> lane) & 1ull) T.hits[out0 + cnt++] = cj[q];
    } else {
      unsigned long long mine = 0;
      for (int q = 0; q < m; ++q) {
        const bool hit = valid && pair_hit(o, v, cp[q], t_min, t_max);
        const unsigned long long bm = __ballot(hit);
        mine = (lane == q) ? bm : mine;
        cnt += hit ? 1 : 0;
      }
      if (k < e) T.masks[k] = mine;
    }
    __syncthreads();
  }
  if (!FILL && valid) {
    T.count[r] = cnt;
    atomicMax(T.max_hits, (unsigned long long)cnt);
  }
}

// ============================================================== per-ray field

struct MergeTables {
  double node[kMaxD + 1], wgt[kMaxD + 1];          // Gauss-Legendre on [0, 1], D + 1 points
  double leg2pow[kMaxD + 1][kMaxD + 1];            // P~_j(u) = sum_d leg2pow[j][d] u^d (shifted Legendre)
  double err_c;  // rounding bound of the merge test per exact piece, relative to the mean square
};

struct FieldArgs {
  // rays
  const double* o;
  const double* v;
  int64_t n_rays;
  double t_min, t_max;
  const float* tr;         // optional per-ray [t_min, t_max] (batches)
  const uint32_t* order;   // optional processing order of the rays (longest first)
  // hits
  const int64_t* hit_count;
  const int64_t* hit_off;
  const uint32_t* hits;
  int64_t hit_slots;  // > 0: ray r's hits at hits[r * hit_slots ...] (single-pass gathering)
  // particles (Morton order)
  const float4* pos4;
  const float* val;
  const int32_t* orig;
  // table
  const void* theta;    // [n_lut][P], stored as tab_fmt
  const void* shat;     // [n_lut][P][D+1], stored as tab_fmt
  int tab_fmt;          // table storage: 0 float64, 1 float32, 2 bfloat16, 3 binary16
  int trans_axis;       // >= 0: pair amplitude value * ((o + t_chi v - chi) . e_axis) / h
  MethodConsts mc;
  MergeTables mt;
  // scheduling
  unsigned int* queue;
  int rays_per_wg;      // > 0: each work-group of a launch takes at most this many rays
  int64_t lds_bytes;    // dynamic LDS of the launch (per-ray layouts up to this size live there)
  int nj;               // jump values per hit
  char* slab;           // per-work-group global storage
  int64_t slab_stride;  // bytes per work-group
  int64_t max_knots;    // largest knot count of any ray (sizes the slab)
  int64_t slab_jmp;     // offset of the jump rows in a work-group's slab
  int64_t slab_scratch; // offset of the sort scratch in a work-group's slab
  int64_t slab_store;   // offset of the whole per-ray layout in a work-group's slab
  uint32_t* flags;
  unsigned long long* counters;  // [0] merged pieces (bump), [1] exact pieces (bump), [2] pieces total,
                                 // [3] rays in device memory, [4] rays with jump rows in device memory,
                                 // [5] rays with jump rows and sort scratch in device memory
  // approx outputs (staging, bump-allocated)
  int64_t out_cap;
  float* st_t0;
  float* st_t1;
  float* st_coef;
  int64_t* ray_out;     // [n][2]: staging offset, count
  float* ray_peak;
  // exact mode
  int exact;
  int64_t exact_cap;
  int64_t* ex_t;
  int64_t* ex_end;
  int64_t* ex_coef;
  int64_t* ray_ex;      // [n][2]
  const int64_t* knot_off;  // [n]
  int64_t knot_cap;
  int64_t* kn_t;
  int32_t* kn_pid;
  int32_t* kn_kidx;
  // render
  const float* tf;
  int tf_n;
  float tf_vmin, tf_vmax;
  double tf_step;
  float* rgba;
};

// A merged interval of exact pieces, held as what the merge test needs: the moments of the exact
// field F about the interval's start and its energy (F in units of sigma, t in length quanta), from
// which the L2 projection onto polynomials of degree <= D and its residual follow.  After the merge,
// finalize_node() replaces the moments by the projection's power coefficients in u = (t - a) / (b - a).
template <int D>
struct Node {
  uint32_t a, b;    // [a, b] in length quanta, relative to the ray's first knot
  int32_t n;        // exact pieces in it
  int32_t pad;
  double m[D + 1];  // m_i = int_a^b F(t) (t - a)^i dt; after finalize_node: power coefficients (world units)
  double e;         // int_a^b F(t)^2 dt
};

__device__ __forceinline__ int64_t rint_i64(double x, uint32_t* flags) {
  if (!(fabs(x) < 4.6e18)) {
    atomicOr(flags, kFlagCoefRange);
    return 0;
  }
  return (int64_t)rint(x);
}

template <int D>
__device__ __forceinline__ void taylor_shift(uint64_t* a, uint32_t delta) {
  const uint64_t dd = (uint64_t)delta;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = D - 1; j >= i; --j) a[j] += a[j + 1] * dd;
}

// Binomial coefficients C(n, k), n, k <= kMaxD, from a compile-time table (the loops that use them
// are unrolled, so every use folds to a constant)
struct BinomTable {
  uint64_t v[kMaxD + 1][kMaxD + 1];
};
constexpr BinomTable make_binom_table() {
  BinomTable t{};
  for (int n = 0; n <= kMaxD; ++n) {
    t.v[n][0] = 1;
    for (int k = 1; k <= n; ++k) t.v[n][k] = t.v[n - 1][k - 1] + (k <= n - 1 ? t.v[n - 1][k] : 0);
  }
  return t;
}
__device__ __forceinline__ uint64_t binom_c(int n, int k) {
  constexpr BinomTable T = make_binom_table();
  return T.v[n][k];
}

// Rows of jump values stored per hit: one row of D orders for each knot pair +-theta_k, plus the
// middle knot for even K.
__host__ __device__ inline int jump_values_per_hit(int P, int even_k, int D) { return (P + even_k) * D; }

// A row of the table of Sec. 3.1 as stored on the device: float64, or narrower (float32, bfloat16,
// binary16) for the storage-precision study; every stored value widens exactly to float64.
struct TabRef {
  const void* base;
  int fmt;      // 0 float64, 1 float32, 2 bfloat16, 3 binary16
  int64_t off;  // first element of the row
  __device__ __forceinline__ double operator[](int i) const {
    const int64_t k = off + i;
    switch (fmt) {
      case 1: return (double)static_cast<const float*>(base)[k];
      case 2: return (double)__uint_as_float((uint32_t)static_cast<const uint16_t*>(base)[k] << 16);
      case 3: return (double)(float)static_cast<const _Float16*>(base)[k];
      default: return static_cast<const double*>(base)[k];
    }
  }
};

// Quantized jump coefficients of all knots of one particle on one ray (Eq. quantized jumps from
// the table, Sec. 4.3, with the integer closure of App. A.3), written as rows of orders 1..D
// (order 0 never jumps):
//   row k-1, k = 1..P: the knot at +theta_k; the knot at -theta_k mirrors it (even orders negated);
//   odd K: row 0 is the knot at +theta_1, whose odd orders come from the closure;
//   even K: row P is the middle knot (odd orders from the closure, even orders zero).
// srow: the hit's table row, s-hat[m][d] (projection jump of order d at +theta_{m+1}, Sec. 3.1) at
// srow[m (D + 1) + d].  The knot pairs are visited one at a time (their table jumps read from
// memory as they are needed), keeping only the closure sums live; the closure's polynomial sums
// in the knot offsets are evaluated by Horner's rule with the 32-bit offset as multiplier.
// Computed once per hit, so the scans over the sorted knots only look values up.  Returns false if
// a quantized coefficient left the int64 range.
template <int D>
__device__ bool hit_jumps(const MethodConsts& mc, TabRef srow, double base, double u, const int32_t* off,
                          uint64_t* rows) {
  const int P = mc.P;
  constexpr int ND = (D + 1) / 2;  // odd orders 1, 3, ...
  uint64_t acc[ND];
#pragma unroll
  for (int i = 0; i < ND; ++i) acc[i] = 0;
  bool ok = true;
  // left[j]: jump of order j at -theta_{m+1} = (-1)^(j+1) times the table jump at +theta_{m+1}
  auto table_left = [&](int m, uint64_t* left) {
    double p = 1.0;
#pragma unroll
    for (int d = 1; d <= D; ++d) {
      p = p * u;
      const double scale = base * p;
      const double x = srow[m * (D + 1) + d] * scale;
      ok = ok && (fabs(x) < 4.6e18);
      const uint64_t j = (fabs(x) < 4.6e18) ? (uint64_t)(int64_t)rint(x) : 0ull;
      left[d] = (d % 2 == 0) ? (uint64_t)0 - j : j;
    }
  };
  // knot pairs whose table jumps enter the closure sums directly: all of them for even K
  // (middle knot), m = 1..P-1 for odd K (the pair +-theta_1 is solved for below)
#pragma unroll 1
  for (int m = 0; m < P; ++m) {
    if (m == 0 && !mc.even_k) continue;
    uint64_t left[D + 1];
    table_left(m, left);
    const uint64_t o = (uint64_t)(uint32_t)off[m];
#pragma unroll
    for (int d = 1; d <= D; d += 2) {
      // even K: sum_{j=d..D} C(j,d) a_{-m,j} o^(j-d); odd K: a_{-m,d} + sum_{j>d} (same terms)
      uint64_t t = binom_c(D, d) * left[D];
#pragma unroll
      for (int jj = D - 1; jj >= d; --jj) t = t * o + binom_c(jj, d) * left[jj];
      acc[d / 2] += t;
    }
#pragma unroll
    for (int d = 1; d <= D; ++d) rows[m * D + d - 1] = (d % 2 == 0) ? (uint64_t)0 - left[d] : left[d];
  }
  if (mc.even_k) {
    // middle knot: a_0d = -2 sum_m sum_{j=d..D} C(j,d) a_{-m,j} o_m^(j-d), odd d
#pragma unroll
    for (int d = 1; d <= D; ++d) rows[P * D + d - 1] = (d % 2 == 1) ? (uint64_t)0 - 2 * acc[d / 2] : 0ull;
    return ok;
  }
  // odd K, knots -1 and +1: odd d in decreasing order
  //   a_{-1,d} = -sum_{m=2..P} a_{-m,d} - sum_{j=d+1..D} C(j,d) sum_{m=1..P} a_{-m,j} o_m^(j-d)
  // (for m = 1 only even j come from the table: odd j use the values already solved)
  uint64_t left[D + 1];
  table_left(0, left);
  const uint64_t o = (uint64_t)(uint32_t)off[0];
#pragma unroll
  for (int d = (D % 2 == 1 ? D : D - 1); d >= 1; d -= 2) {
    uint64_t t = 0;
#pragma unroll
    for (int jj = D; jj > d; --jj) t = t * o + binom_c(jj, d) * left[jj];
    t = t * o + acc[d / 2];
    left[d] = (uint64_t)0 - t;
  }
  // row 0: the knot at +theta_1, a_{1,d} = (-1)^(d+1) a_{-1,d}
#pragma unroll
  for (int d = 1; d <= D; ++d) rows[d - 1] = (d % 2 == 0) ? (uint64_t)0 - left[d] : left[d];
  return ok;
}

// Leaf of the merge: one exact piece [ta, tb) whose field is sum_d a_d (t - ta)^d (coef, wrap-around
// integers read as signed).  Moments and energy by (D + 1)-point Gauss-Legendre quadrature, exact
// for the degree <= 2D integrands.
template <int D>
__device__ __forceinline__ Node<D> make_leaf(const MergeTables& mt, uint32_t ta, uint32_t tb, const uint64_t* coef) {
  #pragma clang fp contract(fast)  // merge arithmetic: fused multiply-adds (no exact key depends on it)
  Node<D> n;
  n.a = ta;
  n.b = tb;
  n.n = 1;
  n.pad = 0;
  const double L = (double)((int64_t)tb - (int64_t)ta);
  double c[D + 1];
#pragma unroll
  for (int d = 0; d <= D; ++d) c[d] = (double)(int64_t)coef[d];
#pragma unroll
  for (int i = 0; i <= D; ++i) n.m[i] = 0.0;
  n.e = 0.0;
#pragma unroll
  for (int g = 0; g <= D; ++g) {
    const double x = L * mt.node[g];
    double f = c[D];
#pragma unroll
    for (int d = D - 1; d >= 0; --d) f = f * x + c[d];
    const double wf = mt.wgt[g] * L * f;
    n.e += wf * f;
    double p = wf;
#pragma unroll
    for (int i = 0; i <= D; ++i) {
      n.m[i] += p;
      p *= x;
    }
  }
  return n;
}

// Union of adjacent nodes A = [a, b] and B = [b, c]: B's moments moved from b to a
// (m_i <- sum_j C(i, j) (b - a)^(i - j) m_j, as repeated synthetic steps) plus A's.
template <int D>
__device__ __forceinline__ Node<D> combine(const Node<D>& A, const Node<D>& B) {
  #pragma clang fp contract(fast)  // merge arithmetic: fused multiply-adds (no exact key depends on it)
  Node<D> U;
  U.a = A.a;
  U.b = B.b;
  U.n = A.n + B.n;
  U.pad = 0;
  const double dl = (double)((int64_t)B.a - (int64_t)A.a);
  double m[D + 1];
#pragma unroll
  for (int i = 0; i <= D; ++i) m[i] = B.m[i];
#pragma unroll
  for (int k = 1; k <= D; ++k)
#pragma unroll
    for (int i = D; i >= k; --i) m[i] += dl * m[i - 1];
#pragma unroll
  for (int i = 0; i <= D; ++i) U.m[i] = A.m[i] + m[i];
  U.e = A.e + B.e;
  return U;
}

// Legendre moments lam_j = int_0^1 f(u) P~_j(u) du of the node's field on u = (t - a) / (b - a) and
// its mean square int_0^1 f^2 du.
template <int D>
__device__ __forceinline__ void node_moments(const MergeTables& mt, const Node<D>& n, double* lam, double* ms) {
  #pragma clang fp contract(fast)  // merge arithmetic: fused multiply-adds (no exact key depends on it)
  const double inv = 1.0 / (double)((int64_t)n.b - (int64_t)n.a);
  double mh[D + 1];
  double p = inv;
#pragma unroll
  for (int i = 0; i <= D; ++i) {
    mh[i] = n.m[i] * p;
    p *= inv;
  }
#pragma unroll
  for (int j = 0; j <= D; ++j) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i <= j; ++i) s += mt.leg2pow[j][i] * mh[i];
    lam[j] = s;
  }
  *ms = n.e * inv;
}

// Merge test: the mean square of F minus its projection, int_0^1 f^2 - sum_j (2j + 1) lam_j^2, plus
// a bound on the rounding of that difference, is within thr2 = (tol * peak)^2 (units of sigma).  The
// bound makes every accepted interval valid; near the threshold the test may refuse a union that
// exact arithmetic would accept.
template <int D>
__device__ __forceinline__ bool passes(const MergeTables& mt, const Node<D>& n, double thr2) {
  #pragma clang fp contract(fast)  // merge arithmetic: fused multiply-adds (no exact key depends on it)
  double lam[D + 1], ms;
  node_moments<D>(mt, n, lam, &ms);
  double q = 0.0;
#pragma unroll
  for (int j = 0; j <= D; ++j) q += (2.0 * j + 1.0) * lam[j] * lam[j];
  const double bound = ((double)n.n * (D + 2) + 16.0) * mt.err_c * ms;
  return (ms - q) + bound <= thr2;
}

// Replace the node's moments by the power coefficients (world units, sigma applied) of the
// projection in u = (t - a) / (b - a): c_d = sigma sum_j (2j + 1) lam_j leg2pow[j][d].
template <int D>
__device__ __forceinline__ void finalize_node(const MergeTables& mt, Node<D>& n, double sigma) {
  #pragma clang fp contract(fast)  // merge arithmetic: fused multiply-adds (no exact key depends on it)
  double lam[D + 1], ms;
  node_moments<D>(mt, n, lam, &ms);
#pragma unroll
  for (int d = 0; d <= D; ++d) {
    double s = 0.0;
#pragma unroll
    for (int j = d; j <= D; ++j) s += (2.0 * j + 1.0) * lam[j] * mt.leg2pow[j][d];
    n.m[d] = sigma * s;
  }
}

__device__ __forceinline__ uint32_t key_slot(uint64_t key) { return (uint32_t)key >> 3; }
__device__ __forceinline__ int key_kidx(uint64_t key) { return (int)((uint32_t)key & 7u); }

// Scan state carried between threads.
template <int D>
struct Agg {
  uint64_t a[D + 1];
  uint32_t t;  // position of the last knot (relative to the ray's first knot)
  int32_t valid;
};

template <int D>
__device__ __forceinline__ void agg_combine(const Agg<D>& x, const Agg<D>& y, Agg<D>& out) {
  if (!x.valid) {
    out = y;
    return;
  }
  if (!y.valid) {
    out = x;
    return;
  }
  out.t = y.t;
  out.valid = 1;
  uint64_t s[D + 1];
#pragma unroll
  for (int d = 0; d <= D; ++d) s[d] = x.a[d];
  taylor_shift<D>(s, y.t - x.t);
#pragma unroll
  for (int d = 0; d <= D; ++d) out.a[d] = s[d] + y.a[d];
}

template <int D, int NT>
struct Shared {
  union {                          // never live together: LDS is the ray layout's capacity
    Agg<D> hs[NT / 64];  // the waves' totals in the scan of the thread aggregates
    float part[NT][4];  // compositing partials (render, at the end)
    uint32_t sort_tab[384 * (NT / 64)];  // slots and digit counts of the knot sort
  };
  uint32_t rtab[32 * (NT / 64)];  // radix sort tables
  int64_t wtot[NT / 64];
  unsigned long long peak;
  int64_t ray;
  int64_t base_out, base_ex;
  long long t_lo, t_hi;  // range of the ray's knot positions (length quanta)
};

// Per-ray storage carved from LDS or from the work-group's global slab.
struct RayStore {
  uint64_t* kkey;
  uint64_t* kkey2;  // radix sort scratch
  uint64_t* jmp;    // [nh][nj] jump rows of every hit (hit_jumps)
  int nj;
  int32_t* ccnt;   // [n_chunks] nodes emitted per chunk
  int32_t* chead;  // [n_chunks] first live node per chunk
  int32_t* gfirst; // [n_chunks] group first node ref
  int32_t* glast;  // [n_chunks] group last node ref
};

__host__ __device__ inline int64_t align8(int64_t x) { return (x + 7) & ~int64_t(7); }

// The sorted knot keys are stored with one unused slot after every 16 (position i at
// kpad(i)), so that threads walking consecutive 16-knot chunks read different LDS banks.
__host__ __device__ inline int64_t kpad(int64_t i) { return i + (i >> 4); }
__host__ __device__ inline int64_t kpad_size(int64_t n) { return n + (n >> 4) + 1; }
__device__ __forceinline__ int kpad32(int i) { return i + (i >> 4); }

// bytes of the per-ray layout for nh hits and nk knots, with or without the jump rows and the
// sort scratch (those two can live in the work-group's device-memory slab instead)
__host__ __device__ inline int64_t ray_store_bytes(int64_t nh, int64_t nk, int nj, bool with_jumps,
                                                   bool with_scratch = true) {
  const int64_t nc = (nk + kChunk - 1) / kChunk;
  return (with_scratch ? 16 : 8) * kpad_size(nk) + (with_jumps ? 8 * (int64_t)nj * nh : 0) + 4 * align8(4 * nc);
}

// Placement tiers of a ray's layout: 0 all in LDS; 1 jump rows in device memory; 2 jump rows and
// sort scratch in device memory; 3 everything in device memory.
__host__ __device__ inline int ray_tier(int64_t nh, int64_t nk, int nj, int64_t lds_bytes) {
  if (ray_store_bytes(nh, nk, nj, true, true) <= lds_bytes) return 0;
  if (ray_store_bytes(nh, nk, nj, false, true) <= lds_bytes) return 1;
  if (ray_store_bytes(nh, nk, nj, false, false) <= lds_bytes) return 2;
  return 3;
}

// jmp_ext / scratch_ext: jump rows / sort scratch kept in device memory instead of in this layout
__device__ inline RayStore carve(char* p, int64_t nh, int64_t nk, int nj, uint64_t* jmp_ext,
                                 uint64_t* scratch_ext = nullptr) {
  RayStore s;
  const int64_t nc = (nk + kChunk - 1) / kChunk;
  s.nj = nj;
  s.kkey = (uint64_t*)p;
  p += 8 * kpad_size(nk);
  if (scratch_ext) {
    s.kkey2 = scratch_ext;
  } else {
    s.kkey2 = (uint64_t*)p;
    p += 8 * kpad_size(nk);
  }
  if (jmp_ext) {
    s.jmp = jmp_ext;
  } else {
    s.jmp = (uint64_t*)p;
    p += 8 * (int64_t)nj * nh;
  }
  s.ccnt = (int32_t*)p;
  p += align8(4 * nc);
  s.chead = (int32_t*)p;
  p += align8(4 * nc);
  s.gfirst = (int32_t*)p;
  p += align8(4 * nc);
  s.glast = (int32_t*)p;
  return s;
}

// Jump coefficients a_0..a_D of the knot named by a sort key, from its hit's rows.
template <int D>
__device__ __forceinline__ void jump_of(const MethodConsts& mc, const RayStore& S, uint64_t key, uint64_t* a) {
  const uint32_t slot = key_slot(key);
  const int k = key_kidx(key) - mc.P;
  const int row = (k == 0) ? mc.P : (k < 0 ? -k : k) - 1;
  const uint64_t* v = S.jmp + ((int)slot * S.nj + row * D);
  a[0] = 0;
#pragma unroll
  for (int d = 1; d <= D; ++d) a[d] = (k < 0 && (d % 2 == 0)) ? (uint64_t)0 - v[d - 1] : v[d - 1];
}

// The exact-mode knot list's second sort (canonical order).
template <int NT>
__device__ __forceinline__ void sort_canonical(uint64_t* a, uint64_t* tmp, int n, int nbits, uint32_t* tab, int tid) {
  radix_sort_u64<NT, false>(a, tmp, n, 0, nbits, tab, tid);
}

// Process one ray with all threads of the work-group.
template <int D, bool RENDER, int NT>
__device__ __forceinline__ void process_ray(const FieldArgs& A, Shared<D, NT>& sh, const RayStore& S, Node<D>* nodes,
                                            int64_t r,
                            int64_t nh) {
  // opaque to the optimiser, so that per-thread addresses are not hoisted out of the ray loop and
  // kept live in registers across every phase
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int K = A.mc.K, P = A.mc.P;
  const int nk = (int)nh * (K + 1);  // at most 1023 * 256 (checked on the host)
  const int64_t hoff = A.hit_slots ? r * A.hit_slots : A.hit_off[r];
  double o[3], v[3];
  for (int k = 0; k < 3; ++k) {
    o[k] = A.o[3 * r + k];
    v[k] = A.v[3 * r + k];
  }
  if (tid == 0) {
    sh.t_lo = 0x7fffffffffffffffll;
    sh.t_hi = -0x7fffffffffffffffll - 1;
  }
  __syncthreads();
  // ---- per-hit records (Sec. 4.3: quantized positions and jumps); the hit order does not matter:
  // knots at equal positions add exactly, so the field, its pieces and the merge are independent
  // of it.  The position t0 and offsets o_1..o_P of hit s are parked in the first words of the
  // hit's own key span until the keys replace them.
  const double tau = A.mc.tau, sigma = A.mc.sigma;
  int32_t* park = reinterpret_cast<int32_t*>(S.kkey);
  const int span32 = 2 * (K + 1);
  long long my_lo = 0x7fffffffffffffffll, my_hi = -0x7fffffffffffffffll - 1;
#pragma unroll 1
  for (int s = tid; s < (int)nh; s += NT) {
    const uint32_t j = A.hits[hoff + s];
    const float4 p = A.pos4[j];
    const float vj = A.val[j];
    const double dxx = (double)p.x - o[0], dxy = (double)p.y - o[1], dxz = (double)p.z - o[2];
    const double cx = dxy * v[2] - dxz * v[1];
    const double cy = dxz * v[0] - dxx * v[2];
    const double cz = dxx * v[1] - dxy * v[0];
    const double z = (double)p.w;
    const double lam2 = (cx * cx + cy * cy + cz * cz) / (z * z);
    const double tchi = dxx * v[0] + dxy * v[1] + dxz * v[2];
    const double lam = sqrt(lam2);
    int li = (int)floor(lam * (double)A.mc.n_lut / kSupport);
    li = li < 0 ? 0 : (li > A.mc.n_lut - 1 ? A.mc.n_lut - 1 : li);
    // the table row: knots now, projection jumps as hit_jumps needs them
    const TabRef trow{A.theta, A.tab_fmt, (int64_t)li * P};
    const TabRef srow{A.shat, A.tab_fmt, (int64_t)li * P * (D + 1)};
    double th[kMaxP];
#pragma unroll
    for (int m = 0; m < kMaxP; ++m) th[m] = (m < P) ? trow[m] : 0.0;
    // positions in 64-bit integers, knot offsets (at most q h / tau) in 32 bits
    const double t0d = rint(tchi / tau);
    bool bad = !(fabs(t0d) < 4.0e18);
    const long long t0 = bad ? 0 : (long long)t0d;
    int32_t offs[kMaxP] = {0, 0, 0};
#pragma unroll
    for (int m = 0; m < kMaxP; ++m) {
      if (m >= P) continue;
      const double od = rint(z * th[m] / tau);
      if (!(od < 2.0e9)) bad = true;
      offs[m] = bad ? 0 : (int32_t)od;
    }
    if (bad) atomicOr(A.flags, kFlagPosRange);
    park[s * span32] = (int32_t)(uint32_t)(unsigned long long)t0;
    park[s * span32 + 1] = (int32_t)(uint32_t)((unsigned long long)t0 >> 32);
#pragma unroll
    for (int m = 0; m < kMaxP; ++m)
      if (m < P) park[s * span32 + 2 + m] = offs[m];
    // transverse gradient field: the pair's amplitude carries its perpendicular offset along the
    // axis, m = (t_chi v_a - dx_a) / h
    double amp = (double)vj;
    if (A.trans_axis >= 0) {
      const double va = A.trans_axis == 0 ? v[0] : (A.trans_axis == 1 ? v[1] : v[2]);
      const double da = A.trans_axis == 0 ? dxx : (A.trans_axis == 1 ? dxy : dxz);
      amp = amp * ((tchi * va - da) / z);
    }
    const double base = amp / (sigma * (z * z * z));
    const double u = tau / z;
    if (!hit_jumps<D>(A.mc, srow, base, u, offs, S.jmp + s * S.nj)) atomicOr(A.flags, kFlagCoefRange);
    const int32_t oP = (P == 1) ? offs[0] : ((P == 2) ? offs[1] : offs[2]);
    my_lo = min(my_lo, t0 - oP);
    my_hi = max(my_hi, t0 + oP);
  }
  atomicMin(&sh.t_lo, my_lo);
  atomicMax(&sh.t_hi, my_hi);
  __syncthreads();
  // Inside the ray, positions are relative to its first knot, t_lo: unsigned 32-bit keys, nodes and
  // differences (the knots of one ray must span less than 2^32 quanta, checked here); absolute
  // positions t_lo + t only at the outputs.
  const long long t_lo = sh.t_lo;
  if (tid == 0 && !(sh.t_hi - t_lo < 4294967295ll)) atomicOr(A.flags, kFlagPosRange);
  auto key_t = [](uint64_t key) { return (uint32_t)(key >> 32); };
  // ---- knot keys: (position - t_lo) in the high half, (slot, kidx) in the low half; kidx = k + P
  // for the knot at t0 + sign(k) o_|k|, laid out slot-major so that the stable sort leaves equal
  // positions in (slot, kidx) order.  Each thread rewrites the spans of the hits it parked.
  for (int s = tid; s < (int)nh; s += NT) {
    const long long t0 = (long long)(((unsigned long long)(uint32_t)park[s * span32 + 1] << 32) |
                                     (unsigned long long)(uint32_t)park[s * span32]);
    int32_t o3[kMaxP];
#pragma unroll
    for (int m = 0; m < kMaxP; ++m) o3[m] = (m < P) ? park[s * span32 + 2 + m] : 0;
    for (int kidx = 0; kidx <= 2 * P; ++kidx) {
      const int k = kidx - P;
      if (k == 0 && !A.mc.even_k) continue;
      int32_t om = 0;
#pragma unroll
      for (int m = 0; m < kMaxP; ++m) om = (m == (k < 0 ? -k : k) - 1) ? o3[m] : om;
      const long long t = t0 + (k < 0 ? -om : om);
      const int slotk = A.mc.even_k ? kidx : (k < 0 ? kidx : kidx - 1);
      S.kkey[s * (K + 1) + slotk] = ((uint64_t)(uint32_t)(t - t_lo) << 32) | ((uint64_t)s << 3) | (uint64_t)kidx;
    }
  }
  __syncthreads();
  {
    // the position bits of the ray's range (at least one), 8 per pass
    const uint32_t range = (uint32_t)(sh.t_hi - t_lo);
    const int nbits = range ? 32 - __clz(range) : 1;
    radix_sort_u64_d8<NT, true>(S.kkey, S.kkey2, (int)nk, 32, nbits, sh.sort_tab, tid);
  }
  // ---- thread ranges of chunks
  const int n_chunks = (nk + kChunk - 1) / kChunk;
  const int per = (n_chunks + NT - 1) / NT;
  const int c_lo = min(tid * per, n_chunks), c_hi = min(c_lo + per, n_chunks);
  const int k_lo = c_lo * kChunk, k_hi = min(c_hi * kChunk, nk);
  // ---- pass A: aggregate of this thread's knots
  Agg<D> agg_mine;
  {
    Agg<D> g;
    g.valid = 0;
    g.t = 0;
    for (int d = 0; d <= D; ++d) g.a[d] = 0;
    for (int i = k_lo; i < k_hi; ++i) {
      const uint64_t key = S.kkey[kpad32(i)];
      const uint32_t t = key_t(key);
      uint64_t jmp[D + 1];
      jump_of<D>(A.mc, S, key, jmp);
      if (g.valid) taylor_shift<D>(g.a, (uint32_t)(t - g.t));
      for (int d = 0; d <= D; ++d) g.a[d] += jmp[d];
      g.t = t;
      g.valid = 1;
    }
    agg_mine = g;
  }
  // scan of the thread aggregates in thread order (exact integers: any grouping gives the same
  // states): inclusive within each wave by lane shuffles, then the totals of the earlier waves
  // through LDS; a thread's carry is the inclusive aggregate of the thread before it
  Agg<D> carry;
  {
    const int lane = tid & 63, wv = tid >> 6;
    Agg<D> x = agg_mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      Agg<D> y;
#pragma unroll
      for (int d = 0; d <= D; ++d) y.a[d] = __shfl_up(x.a[d], o, 64);
      y.t = __shfl_up(x.t, o, 64);
      y.valid = __shfl_up(x.valid, o, 64);
      if (lane >= o) {
        Agg<D> res;
        agg_combine<D>(y, x, res);
        x = res;
      }
    }
    if (lane == 63) sh.hs[wv] = x;
    __syncthreads();
    Agg<D> pre;
    pre.valid = 0;
    pre.t = 0;
#pragma unroll
    for (int d = 0; d <= D; ++d) pre.a[d] = 0;
    for (int ww = 0; ww < wv; ++ww) {
      Agg<D> res;
      agg_combine<D>(pre, sh.hs[ww], res);
      pre = res;
    }
    Agg<D> below;  // inclusive aggregate of the previous lane of this wave
#pragma unroll
    for (int d = 0; d <= D; ++d) below.a[d] = __shfl_up(x.a[d], 1, 64);
    below.t = __shfl_up(x.t, 1, 64);
    below.valid = __shfl_up(x.valid, 1, 64);
    if (lane == 0) carry = pre;
    else agg_combine<D>(pre, below, carry);
  }
  // ---- pass B: peak over piece starts, tail check, piece counts
  if (tid == 0) sh.peak = 0;
  __syncthreads();
  unsigned long long pk = 0;
  int64_t npieces = 0;
  {
    Agg<D> st = carry;
    for (int i = k_lo; i < k_hi; ++i) {
      const uint64_t key = S.kkey[kpad32(i)];
      const uint32_t t = key_t(key);
      uint64_t jmp[D + 1];
      jump_of<D>(A.mc, S, key, jmp);
      if (st.valid) taylor_shift<D>(st.a, (uint32_t)(t - st.t));
      for (int d = 0; d <= D; ++d) st.a[d] += jmp[d];
      st.t = t;
      st.valid = 1;
      const bool last = (i + 1 == nk);
      if (!last && key_t(S.kkey[kpad32(i + 1)]) != t) {
        const int64_t a0 = (int64_t)st.a[0];
        const unsigned long long m = (unsigned long long)(a0 < 0 ? -a0 : a0);
        pk = pk > m ? pk : m;
        ++npieces;
      }
      if (last) {
        bool zero = true;
        for (int d = 0; d <= D; ++d) zero = zero && (st.a[d] == 0);
        if (!zero) atomicOr(A.flags, kFlagTail);
      }
    }
  }
  atomicMax(&sh.peak, pk);
  // exclusive scan of piece counts (exact-mode positions)
  int64_t run = 0;
  const int64_t ex_first = block_excl_scan_i64<NT>(npieces, sh.wtot, tid, &run);
  const double peak = sigma * (double)(int64_t)sh.peak;
  if (tid == 0) {
    if (A.exact) {
      sh.base_ex = (int64_t)atomicAdd(&A.counters[1], (unsigned long long)run);
      A.ray_ex[2 * r] = sh.base_ex;
      A.ray_ex[2 * r + 1] = run;
    }
    atomicAdd(&A.counters[2], (unsigned long long)run);
  }
  __syncthreads();
  // ---- pass C: exact pieces -> leaves -> greedy merge within chunks -> nodes.  A chunk's first
  // node lives in the sort scratch (free from here to the end; most chunks keep at most one node
  // after the merge, and for rays laid out in LDS the junction tree and the output then read them
  // from LDS), the others in the work-group's slab.
  const bool first_in_scratch = (int64_t)sizeof(Node<D>) * n_chunks <= 8 * kpad_size(nk);
  Node<D>* const first_nodes = reinterpret_cast<Node<D>*>(S.kkey2);
  auto node = [&](int32_t id) -> Node<D>& {
    return (first_in_scratch && id % kChunk == 0) ? first_nodes[id / kChunk] : nodes[id];
  };
  const double tol = A.mc.merge_tol;
  const double pk_s = (double)sh.peak;  // the peak in units of sigma
  const double thr2 = (tol * pk_s) * (tol * pk_s);
  {
    Agg<D> st = carry;
    int64_t ex_pos = ex_first;
    int cur_chunk = -1;
    Node<D> cur;
    bool have = false;
    int32_t emitted = 0;
    auto flush = [&](int chunk) {
      if (have) {
        node(chunk * kChunk + emitted) = cur;
        ++emitted;
        have = false;
      }
    };
    for (int c = c_lo; c < c_hi; ++c) S.ccnt[c] = 0;
    for (int i = k_lo; i < k_hi; ++i) {
      const uint64_t key = S.kkey[kpad32(i)];
      const uint32_t t = key_t(key);
      uint64_t jmp[D + 1];
      jump_of<D>(A.mc, S, key, jmp);
      if (st.valid) taylor_shift<D>(st.a, (uint32_t)(t - st.t));
      for (int d = 0; d <= D; ++d) st.a[d] += jmp[d];
      st.t = t;
      st.valid = 1;
      const int chunk = i / kChunk;
      if (chunk != cur_chunk) {
        if (cur_chunk >= 0) {
          flush(cur_chunk);
          S.ccnt[cur_chunk] = emitted;
        }
        cur_chunk = chunk;
        emitted = 0;
      }
      if (i + 1 < nk) {
        const uint32_t tn = key_t(S.kkey[kpad32(i + 1)]);
        if (tn != t) {
          if (A.exact) {
            const int64_t e = sh.base_ex + ex_pos;
            if (e < A.exact_cap) {
              A.ex_t[e] = t_lo + t;
              A.ex_end[e] = t_lo + tn;
              for (int d = 0; d <= D; ++d) A.ex_coef[e * (D + 1) + d] = (int64_t)st.a[d];
            }
          }
          ++ex_pos;
          Node<D> leaf = make_leaf<D>(A.mt, t, tn, st.a);
          if (!have) {
            cur = leaf;
            have = true;
          } else if (tol > 0.0) {
            Node<D> cand = combine<D>(cur, leaf);
            if (passes<D>(A.mt, cand, thr2)) cur = cand;
            else {
              flush(chunk);
              cur = leaf;
              have = true;
            }
          } else {
            flush(chunk);
            cur = leaf;
            have = true;
          }
        }
      }
    }
    if (cur_chunk >= 0) {
      flush(cur_chunk);
      S.ccnt[cur_chunk] = emitted;
    }
  }
  __syncthreads();
  // ---- junction merges across chunk groups (levels 1, 2, 4, ...)
  for (int c = tid; c < n_chunks; c += NT) {
    S.chead[c] = 0;
    const int32_t cn = S.ccnt[c];
    S.gfirst[c] = cn > 0 ? (int32_t)(c * kChunk) : -1;
    S.glast[c] = cn > 0 ? (int32_t)(c * kChunk + cn - 1) : -1;
  }
  __syncthreads();
  if (tol > 0.0) {
    for (int w = 1; w < n_chunks; w <<= 1) {
      for (int L = tid * 2 * w; L < n_chunks; L += NT * 2 * w) {
        const int R = L + w;
        if (R >= n_chunks) continue;
        const int32_t lf = S.gfirst[L], ll = S.glast[L], rf = S.gfirst[R], rl = S.glast[R];
        int32_t nf = lf >= 0 ? lf : rf;
        int32_t nl = rl >= 0 ? rl : ll;
        if (ll >= 0 && rf >= 0) {
          Node<D> cand = combine<D>(node(ll), node(rf));
          if (passes<D>(A.mt, cand, thr2)) {
            node(ll) = cand;
            const int rc = rf / kChunk;
            S.chead[rc] = S.chead[rc] + 1;
            // next live node of group R
            int32_t nxt = -1;
            const int r_end = min(R + w, n_chunks);
            for (int c = rc; c < r_end && nxt < 0; ++c) {
              if (S.chead[c] < S.ccnt[c]) nxt = (int32_t)(c * kChunk + S.chead[c]);
            }
            if (nxt < 0) nl = ll;  // group R became empty
            nf = lf;
          }
        }
        S.gfirst[L] = nf;
        S.glast[L] = nl;
      }
      __syncthreads();
    }
  }
  // ---- live nodes per thread range, in order; their moments become output coefficients
  int64_t mine = 0;
  for (int c = c_lo; c < c_hi; ++c) {
    mine += S.ccnt[c] - S.chead[c];
    for (int32_t q = S.chead[c]; q < S.ccnt[c]; ++q) finalize_node<D>(A.mt, node(c * kChunk + q), sigma);
  }
  int64_t n_live = 0;
  const int64_t live_first = block_excl_scan_i64<NT>(mine, sh.wtot, tid, &n_live);
  if (!RENDER) {
    #pragma clang fp contract(fast)  // output arithmetic: fused multiply-adds
    if (tid == 0) {
      sh.base_out = (int64_t)atomicAdd(&A.counters[0], (unsigned long long)n_live);
      A.ray_out[2 * r] = sh.base_out;
      A.ray_out[2 * r + 1] = n_live;
      A.ray_peak[r] = (float)peak;
    }
    __syncthreads();
    int64_t pos = sh.base_out + live_first;
    for (int c = c_lo; c < c_hi; ++c) {
      for (int32_t q = S.chead[c]; q < S.ccnt[c]; ++q) {
        const Node<D>& nd = node(c * kChunk + q);
        if (pos < A.out_cap) {
          // The piece is delivered on its float32 ends fa, fb: the projection, a polynomial in
          // u = (t - ta) / (tb - ta) over the exact ends, is re-expressed in u' = (t - fa) / (fb - fa)
          // by composing it with u = al + be u' (exact in real arithmetic, float64 here), so that a
          // caller evaluating on the stored ends gets the projection itself.
          const double ta = (double)(t_lo + nd.a) * tau, tb = (double)(t_lo + nd.b) * tau;
          const float fa = (float)ta, fb = (float)tb;
          const double len = (double)((int64_t)nd.b - (int64_t)nd.a) * tau;
          double cu[D + 1];
#pragma unroll
          for (int d = 0; d <= D; ++d) cu[d] = nd.m[d];
          const double al = ((double)fa - ta) / len;
          const double be = ((double)fb - (double)fa) / len;
          double rc[D + 1];
#pragma unroll
          for (int d = 0; d <= D; ++d) rc[d] = 0.0;
          if (fb > fa) {
            // Horner composition: rc = (...(c_D (al + be x) + c_{D-1}) (al + be x) + ...) + c_0
            rc[0] = cu[D];
#pragma unroll
            for (int d = D - 1; d >= 0; --d) {
#pragma unroll
              for (int k = D - d; k >= 1; --k) rc[k] = rc[k] * al + rc[k - 1] * be;
              rc[0] = rc[0] * al + cu[d];
            }
          } else {
            // float32 ends coincide (a piece shorter than their resolution): its value at the start
            double s = cu[D];
#pragma unroll
            for (int d = D - 1; d >= 0; --d) s = s * al + cu[d];
            rc[0] = s;
          }
          A.st_t0[pos] = fa;
          A.st_t1[pos] = fb;
#pragma unroll
          for (int d = 0; d <= D; ++d) A.st_coef[pos * (D + 1) + d] = (float)rc[d];
        }
        ++pos;
      }
    }
    if (A.exact) {
      // sorted knot list in the canonical order (position, particle input index, kidx)
      __syncthreads();
      for (int64_t i = tid; i < nk; i += NT) {
        const uint64_t key = S.kkey[kpad(i)];
        S.kkey2[i] = (key & 0xffffffff00000000ull) | ((uint64_t)(uint32_t)A.orig[A.hits[hoff + key_slot(key)]] << 3) |
                     (uint64_t)key_kidx(key);
      }
      __syncthreads();
      const uint32_t range = (uint32_t)(sh.t_hi - t_lo);
      int nbits = 36;
      while (nbits < 64 && (range >> (nbits - 32)) != 0) nbits += 4;
      sort_canonical<NT>(S.kkey2, S.kkey, (int)nk, nbits, sh.rtab, tid);
      for (int64_t i = tid; i < nk; i += NT) {
        const uint64_t key = S.kkey2[i];
        const int64_t ko = A.knot_off[r] + i;
        if (ko < A.knot_cap) {
          A.kn_t[ko] = t_lo + key_t(key);
          A.kn_pid[ko] = (int32_t)((uint32_t)key >> 3);
          A.kn_kidx[ko] = (int32_t)(key & 7u);
        }
      }
    }
  } else {
    #pragma clang fp contract(fast)  // compositing arithmetic: fused multiply-adds
    // classification and front-to-back compositing.  The samples of the ray's live nodes are
    // numbered in order and split evenly over the threads (merged nodes can be long, so per-node
    // work is uneven); a thread finds its first node by binary search in an index of the nodes'
    // first sample numbers.
    const float vmin = A.tf_vmin, vr = A.tf_vmax - A.tf_vmin;
    const int ntf = A.tf_n;
    const double ray_tmin = A.tr ? (double)A.tr[2 * r] : A.t_min, ray_tmax = A.tr ? (double)A.tr[2 * r + 1] : A.t_max;
    auto sample_count = [&](const Node<D>& nd) -> int64_t {
      const double ta = (double)(t_lo + nd.a) * tau, tb = (double)(t_lo + nd.b) * tau;
      const double a = fmax(ta, ray_tmin), b = fmin(tb, ray_tmax);
      return (b > a) ? (int64_t)fmax(1.0, ceil((b - a) / A.tf_step)) : 0;
    };
    int64_t my_samples = 0;
    for (int c = c_lo; c < c_hi; ++c)
      for (int32_t q = S.chead[c]; q < S.ccnt[c]; ++q) my_samples += sample_count(node(c * kChunk + q));
    int64_t n_samp = 0;
    const int64_t samp_first = block_excl_scan_i64<NT>(my_samples, sh.wtot, tid, &n_samp);
    // node index in the key array (free now; at least 8 bytes per exact piece): first sample
    // number and node slot of each live node
    int32_t* ist = reinterpret_cast<int32_t*>(S.kkey);
    int32_t* iref = ist + n_live;
    {
      int64_t pos = live_first, sp = samp_first;
      for (int c = c_lo; c < c_hi; ++c)
        for (int32_t q = S.chead[c]; q < S.ccnt[c]; ++q) {
          ist[pos] = (int32_t)sp;
          iref[pos] = (int32_t)(c * kChunk + q);
          sp += sample_count(node(c * kChunk + q));
          ++pos;
        }
    }
    // the transfer function is read once per sample: stage it in the jump rows (free now) if it fits
    const float* tfp = A.tf;
    if ((int64_t)ntf * 16 <= 8 * (int64_t)S.nj * nh) {
      float* t = reinterpret_cast<float*>(S.jmp);
      for (int i = tid; i < 4 * ntf; i += NT) t[i] = A.tf[i];
      tfp = t;
    }
    __syncthreads();
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
    const int64_t share = (n_samp + NT - 1) / NT;
    const int64_t g0 = min((int64_t)tid * share, n_samp), g1 = min(g0 + share, n_samp);
    if (g0 < g1) {
      // last node whose first sample number is <= g0 (nodes without samples share the number of
      // the next node, so the search never stops on one of them)
      int64_t lo = 0, hi = n_live - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)ist[mid] <= g0) lo = mid;
        else hi = mid - 1;
      }
      int64_t g = g0;
      for (int64_t n = lo; g < g1; ++n) {
        const Node<D>& nd = node(iref[n]);
        const double ta = (double)(t_lo + nd.a) * tau, tb = (double)(t_lo + nd.b) * tau;
        const double a = fmax(ta, ray_tmin), b = fmin(tb, ray_tmax);
        if (!(b > a)) continue;
        const double Sd = fmax(1.0, ceil((b - a) / A.tf_step));
        const int64_t S_n = (int64_t)Sd;
        const double delta = (b - a) / Sd;
        float cf[D + 1];
        for (int d = 0; d <= D; ++d) cf[d] = (float)nd.m[d];
        const float u0 = (float)((a - ta) / (tb - ta)), du = (float)(delta / (tb - ta));
        const float dl = (float)delta;
        const int64_t first = ist[n];
        const int64_t j1 = min(S_n, g1 - first);
        for (int64_t j = g - first; j < j1; ++j) {
          const float uu = u0 + ((float)j + 0.5f) * du;
          float val = cf[D];
          for (int d = D - 1; d >= 0; --d) val = val * uu + cf[d];
          float x = (val - vmin) / vr * (float)(ntf - 1);
          x = fminf(fmaxf(x, 0.f), (float)(ntf - 1));
          const int i0 = (int)floorf(x);
          const int i1 = min(i0 + 1, ntf - 1);
          const float f = x - (float)i0;
          const float* p0 = tfp + 4 * i0;
          const float* p1 = tfp + 4 * i1;
          const float er = (1.f - f) * p0[0] + f * p1[0];
          const float eg = (1.f - f) * p0[1] + f * p1[1];
          const float eb = (1.f - f) * p0[2] + f * p1[2];
          const float sg = (1.f - f) * p0[3] + f * p1[3];
          const float xx = sg * dl;
          const float frac = (xx == 0.f) ? dl : -expm1f(-xx) / sg;
          C0 += T * er * frac;
          C1 += T * eg * frac;
          C2 += T * eb * frac;
          T *= expf(-xx);
        }
        g = first + j1;
      }
    }
    sh.part[tid][0] = C0;
    sh.part[tid][1] = C1;
    sh.part[tid][2] = C2;
    sh.part[tid][3] = T;
    __syncthreads();
    // ordered tree reduction: (C1, T1) then (C2, T2) = (C1 + T1 C2, T1 T2)
    for (int s = 1; s < NT; s <<= 1) {
      if ((tid % (2 * s)) == 0 && tid + s < NT) {
        const float t1 = sh.part[tid][3];
        sh.part[tid][0] += t1 * sh.part[tid + s][0];
        sh.part[tid][1] += t1 * sh.part[tid + s][1];
        sh.part[tid][2] += t1 * sh.part[tid + s][2];
        sh.part[tid][3] = t1 * sh.part[tid + s][3];
      }
      __syncthreads();
    }
    if (tid == 0) {
      A.rgba[4 * r] = sh.part[0][0];
      A.rgba[4 * r + 1] = sh.part[0][1];
      A.rgba[4 * r + 2] = sh.part[0][2];
      A.rgba[4 * r + 3] = 1.f - sh.part[0][3];
    }
  }
}

// WGS: ray work-groups meant to share a CU (registers capped accordingly; the host sizes the
// dynamic LDS to 1 / WGS of the CU)
template <int D, bool RENDER, int WGS, int NT>
__global__ void __launch_bounds__(NT, WGS) k_field(FieldArgs A) {
  extern __shared__ __align__(16) char lds[];
  __shared__ Shared<D, NT> sh;
  char* slab = A.slab + (int64_t)blockIdx.x * A.slab_stride;
  Node<D>* nodes = (Node<D>*)slab;
  uint64_t* gjmp = (uint64_t*)(slab + A.slab_jmp);
  uint64_t* gscratch = (uint64_t*)(slab + A.slab_scratch);
  char* gstore = slab + A.slab_store;
  for (int taken = 0;; ++taken) {
    // a bounded share per work-group (rays_per_wg > 0) ends the launch early, so that the kernels
    // of other streams get compute units between this stream's launches; the host then launches
    // again until the queue is drained
    if (A.rays_per_wg > 0 && taken == A.rays_per_wg) break;
    if (threadIdx.x == 0) {
      const int64_t q = (int64_t)atomicAdd(A.queue, 1u);
      sh.ray = (q < A.n_rays && A.order) ? (int64_t)A.order[q] : q;
    }
    __syncthreads();
    const int64_t r = sh.ray;
    if (r >= A.n_rays) break;
    const int64_t nh = A.hit_count[r];
    if (nh == 0) {
      if (threadIdx.x == 0) {
        if (RENDER) {
          for (int k = 0; k < 4; ++k) A.rgba[4 * r + k] = 0.f;
        } else {
          A.ray_out[2 * r] = 0;
          A.ray_out[2 * r + 1] = 0;
          A.ray_peak[r] = 0.f;
          if (A.exact) {
            A.ray_ex[2 * r] = 0;
            A.ray_ex[2 * r + 1] = 0;
          }
        }
      }
    } else {
      // the whole layout in LDS if it fits, else the jump rows, then also the sort scratch, then
      // everything in the work-group's device memory (the arithmetic is the same on every path)
      const int64_t nk = nh * (A.mc.K + 1);
      const int tier = ray_tier(nh, nk, A.nj, A.lds_bytes);
      if (tier == 0) {
        // common case, its own inlined copy so that every access compiles to LDS instructions
        const RayStore S = carve(lds, nh, nk, A.nj, nullptr);
        process_ray<D, RENDER, NT>(A, sh, S, nodes, r, nh);
      } else {
        if (threadIdx.x == 0) atomicAdd(&A.counters[tier == 1 ? 4 : (tier == 2 ? 5 : 3)], 1ull);
        const RayStore S = carve(tier < 3 ? lds : gstore, nh, nk, A.nj, tier < 3 ? gjmp : nullptr,
                                 tier == 2 ? gscratch : nullptr);
        process_ray<D, RENDER, NT>(A, sh, S, nodes, r, nh);
      }
    }
    __syncthreads();
  }
}

// ============================================================== finalize (approx mode)

__global__ void k_ray_counts(const int64_t* ray_pair, int64_t n, int64_t* counts) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    counts[r] = ray_pair[2 * r + 1];
}

__global__ void k_copy_pieces(const int64_t* ray_out, const int64_t* final_off, int64_t n, int D1, const float* s0,
                              const float* s1, const float* sc, float* t0, float* t1, float* coef) {
  const int64_t r = (int64_t)blockIdx.x;
  if (r >= n) return;
  const int64_t src = ray_out[2 * r], cnt = ray_out[2 * r + 1], dst = final_off[r];
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
    t0[dst + i] = s0[src + i];
    t1[dst + i] = s1[src + i];
  }
  for (int64_t i = threadIdx.x; i < cnt * D1; i += blockDim.x) coef[dst * D1 + i] = sc[src * D1 + i];
}

__global__ void k_copy_exact(const int64_t* ray_ex, const int64_t* final_off, int64_t n, int D1, const int64_t* s0,
                             const int64_t* s1, const int64_t* sc, int64_t* t0, int64_t* t1, int64_t* coef) {
  const int64_t r = (int64_t)blockIdx.x;
  if (r >= n) return;
  const int64_t src = ray_ex[2 * r], cnt = ray_ex[2 * r + 1], dst = final_off[r];
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
    t0[dst + i] = s0[src + i];
    t1[dst + i] = s1[src + i];
  }
  for (int64_t i = threadIdx.x; i < cnt * D1; i += blockDim.x) coef[dst * D1 + i] = sc[src * D1 + i];
}

__global__ void k_scale_i64(const int64_t* a, int64_t* b, int64_t n, int64_t f) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i] * f;
}

// Hit lists as input indices: ray r's hits from its compact list (hit_slots = 0) or its slots.
__global__ void k_export_hits(const int64_t* hit_off, const uint32_t* hits, int64_t hit_slots, int64_t n,
                              const int32_t* orig, int32_t* ids) {
  for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
    const int64_t b = hit_off[r], e = hit_off[r + 1];
    const uint32_t* src = hit_slots ? hits + r * hit_slots : hits + b;
    for (int64_t i = threadIdx.x; i < e - b; i += blockDim.x) ids[b + i] = orig[src[i]];
  }
}

__global__ void k_set_last(int64_t* off, const int64_t* cnt, int64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) off[n] = (n > 0 ? off[n - 1] + cnt[n - 1] : 0);
}

// ============================================================== host

MergeTables make_merge_tables(int D) {
  MergeTables t{};
  // Gauss-Legendre nodes on [0, 1] with D + 1 points (Newton on P_{D+1})
  const int n = D + 1;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(3.14159265358979323846 * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) {
        p1 = z;
        p0 = 1.0;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    t.node[i] = 0.5 * (z + 1.0);
    t.wgt[i] = 0.5 * 2.0 / ((1.0 - z * z) * dp * dp);
  }
  // shifted Legendre power coefficients: P~_j(u) = sum_k (-1)^(j+k) C(j,k) C(j+k,k) u^k
  auto C = [](int a, int b) {
    double v = 1.0;
    for (int i = 1; i <= b; ++i) v = v * (a - b + i) / i;
    return v;
  };
  for (int j = 0; j <= D; ++j)
    for (int k = 0; k <= D; ++k) t.leg2pow[j][k] = (k <= j) ? (((j + k) % 2) ? -1.0 : 1.0) * C(j, k) * C(j + k, k) : 0.0;
  // Rounding of the merge test.  With |lam_j| <= |f| / sqrt(2j + 1) (Cauchy-Schwarz) and every
  // moment off by at most (pieces) eps |f| (sums of the pieces' terms and of the shifts, whose
  // terms are all bounded by the integral of |F| (t - a)^i), sum_j (2j + 1) lam_j^2 is off by at
  // most 2 sum_j sqrt(2j + 1) S_j (pieces) eps |f|^2, S_j the absolute row sum of P~_j; a factor 2
  // covers the quadrature, the reciprocal and the last subtraction.
  double cd = 0.0;
  for (int j = 0; j <= D; ++j) {
    double sj = 0.0;
    for (int k = 0; k <= j; ++k) sj += std::fabs(t.leg2pow[j][k]);
    cd += std::sqrt(2.0 * j + 1.0) * sj;
  }
  t.err_c = 2.0 * 2.0 * cd * std::ldexp(1.0, -52);
  return t;
}

template <int D, int NT>
size_t shared_static_bytes() {
  return sizeof(Shared<D, NT>);
}

template <int D, bool RENDER, int WGS, int NT>
void launch_field(FieldArgs& A, int grid, size_t lds, hipStream_t st) {
  hip_check(hipFuncSetAttribute((const void*)k_field<D, RENDER, WGS, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds),
            "set lds");
  k_field<D, RENDER, WGS, NT><<<grid, NT, lds, st>>>(A);
  hip_check(hipGetLastError(), "field launch");
}

// Only the configurations whose registers fit without spilling are built (field_cfg_valid).
template <int D, bool RENDER, int CFG>
void launch_field_checked(FieldArgs& A, int grid, size_t lds, hipStream_t st) {
  if constexpr (field_cfg_valid(D, RENDER, CFG))
    launch_field<D, RENDER, field_cfg_wgs(CFG), field_cfg_threads(CFG)>(A, grid, lds, st);
  else
    throw Error(SPH_HOA_E_INTERNAL, "field kernel configuration beyond the degree's limit");
}

template <bool RENDER, int CFG>
void dispatch_field_cfg(int D, FieldArgs& A, int grid, size_t lds, hipStream_t st) {
  switch (D) {
    case 1: launch_field_checked<1, RENDER, CFG>(A, grid, lds, st); break;
    case 2: launch_field_checked<2, RENDER, CFG>(A, grid, lds, st); break;
    case 3: launch_field_checked<3, RENDER, CFG>(A, grid, lds, st); break;
    case 4: launch_field_checked<4, RENDER, CFG>(A, grid, lds, st); break;
    case 5: launch_field_checked<5, RENDER, CFG>(A, grid, lds, st); break;
    case 6: launch_field_checked<6, RENDER, CFG>(A, grid, lds, st); break;
    default: throw Error(SPH_HOA_E_UNSUPPORTED, "degree");
  }
}

template <bool RENDER>
void dispatch_field(int D, int cfg, FieldArgs& A, int grid, size_t lds, hipStream_t st) {
  switch (cfg) {
    case 1: dispatch_field_cfg<RENDER, 1>(D, A, grid, lds, st); break;
    case 2: dispatch_field_cfg<RENDER, 2>(D, A, grid, lds, st); break;
    case 3: dispatch_field_cfg<RENDER, 3>(D, A, grid, lds, st); break;
    case 4: dispatch_field_cfg<RENDER, 4>(D, A, grid, lds, st); break;
    case 5: dispatch_field_cfg<RENDER, 5>(D, A, grid, lds, st); break;
    default: dispatch_field_cfg<RENDER, 6>(D, A, grid, lds, st); break;
  }
}

size_t node_bytes(int D) { return 8 + 8 * (size_t)(D + 3); }

template <int NT>
size_t static_lds_nt(int D) {
  switch (D) {
    case 1: return shared_static_bytes<1, NT>();
    case 2: return shared_static_bytes<2, NT>();
    case 3: return shared_static_bytes<3, NT>();
    case 4: return shared_static_bytes<4, NT>();
    case 5: return shared_static_bytes<5, NT>();
    default: return shared_static_bytes<6, NT>();
  }
}

size_t static_lds(int D, int nt) { return nt == 512 ? static_lds_nt<512>(D) : static_lds_nt<256>(D); }

unsigned blocks_for(int64_t n, int t) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + t - 1) / t, 65536));
}

}  // namespace

// Camera frame of an sph_hoa_camera (float inputs widened to float64).
CamDev make_cam(const sph_hoa_camera* cam) {
  CamDev c{};
  double e[3], la[3], up[3];
  for (int k = 0; k < 3; ++k) {
    e[k] = (double)cam->eye[k];
    la[k] = (double)cam->look_at[k];
    up[k] = (double)cam->up[k];
  }
  auto norm3 = [](double& x, double& y, double& z) {
    const double nn = std::sqrt(x * x + y * y + z * z);
    x = x / nn;
    y = y / nn;
    z = z / nn;
  };
  double fx = la[0] - e[0], fy = la[1] - e[1], fz = la[2] - e[2];
  norm3(fx, fy, fz);
  double rx = fy * up[2] - fz * up[1], ry = fz * up[0] - fx * up[2], rz = fx * up[1] - fy * up[0];
  norm3(rx, ry, rz);
  const double ux = ry * fz - rz * fy, uy = rz * fx - rx * fz, uz = rx * fy - ry * fx;
  const double f[3] = {fx, fy, fz}, rr[3] = {rx, ry, rz}, uu[3] = {ux, uy, uz};
  for (int k = 0; k < 3; ++k) {
    c.eye[k] = e[k];
    c.f[k] = f[k];
    c.r[k] = rr[k];
    c.u[k] = uu[k];
  }
  const double fov = (double)cam->fov_y_deg;
  c.g = std::tan(fov * 3.14159265358979323846 / 180.0 / 2.0);
  c.aspect = (double)cam->width / (double)cam->height;
  c.half = (double)cam->ortho_half_extent;
  c.W = cam->width;
  c.H = cam->height;
  c.ortho = cam->ortho;
  c.t_min = cam->t_min;
  c.t_max = cam->t_max;
  return c;
}

FieldTuner::Key FieldTuner::key_of(int D, bool render, int64_t pairs, int64_t rays, int64_t max_hits) {
  auto lg = [](int64_t x) {
    int b = 0;
    while (x > 1) {
      x >>= 1;
      ++b;
    }
    return b;
  };
  return Key{D, render ? 1 : 0, lg(1 + pairs / std::max<int64_t>(1, rays)), lg(1 + max_hits)};
}

int FieldTuner::chosen(const Key& k) const {
  int best = -1;
  for (int c : kOrder)
    if (field_cfg_valid(k.D, k.render != 0, c)) {
      best = c;  // the first valid candidate while nothing is measured
      break;
    }
  const auto it = table.find(k);
  if (it == table.end()) return best;
  double best_ms = -1.0;
  for (int c : kOrder) {
    if (!field_cfg_valid(k.D, k.render != 0, c)) continue;
    const double v = it->second.ms_per_pair[c];
    if (v >= 0 && (best_ms < 0 || v < best_ms)) {
      best = c;
      best_ms = v;
    }
  }
  return best;
}

int FieldTuner::choose(const Key& k) {
  Entry& e = table[k];
  for (int c : kOrder)
    if (field_cfg_valid(k.D, k.render != 0, c) && e.ms_per_pair[c] < 0) return c;  // measure each candidate once, in order
  return chosen(k);
}

void FieldTuner::begin(const Key& k, int cfg, int64_t pairs, hipStream_t st) {
  Entry& e = table[k];
  const int slot = cfg;
  pending = (e.ms_per_pair[slot] < 0 && pairs > 0);
  if (!pending) return;
  for (auto& v : ev)
    if (!v) hip_check(hipEventCreate(&v), "event");
  pend_key = k;
  pend_slot = slot;
  pend_pairs = pairs;
  hip_check(hipEventRecord(ev[0], st), "event");
}

void FieldTuner::end(hipStream_t st) {
  if (pending) hip_check(hipEventRecord(ev[1], st), "event");
}

void FieldTuner::collect() {
  if (!pending) return;
  pending = false;
  hip_check(hipEventSynchronize(ev[1]), "event sync");
  float ms = 0.f;
  hip_check(hipEventElapsedTime(&ms, ev[0], ev[1]), "elapsed");
  table[pend_key].ms_per_pair[pend_slot] = (double)ms / (double)pend_pairs;
}

FieldTuner::~FieldTuner() {
  for (auto& v : ev)
    if (v) (void)hipEventDestroy(v);
}

void Workspace::collect_timing() {
  if (!timing_pending) return;
  timing_pending = false;
  hip_check(hipEventSynchronize(ev[5]), "event sync");
  float a = 0.f, b = 0.f, c = 0.f;
  hip_check(hipEventElapsedTime(&a, ev[0], ev[1]), "elapsed");
  hip_check(hipEventElapsedTime(&b, ev[2], ev[3]), "elapsed");
  hip_check(hipEventElapsedTime(&c, ev[4], ev[5]), "elapsed");
  ms_gather += (double)a + (double)b;
  ms_field += (double)c;
  ++timed_calls;
}

void run_rays(Index& ix, int64_t n_rays, bool camera, const sph_hoa_camera* cam, const sph_hoa_rays* rays,
              FieldOut& out, hipStream_t st, const sph_hoa_camera* batch, int n_batch, const Index* gathered,
              Workspace* workspace) {
  Workspace& ws = workspace ? *workspace : ix.ws;
  const int D = ix.D, K = ix.K, P = ix.P;
  auto gather_range = std::make_unique<TraceRange>(camera ? "hit gathering (screen tiles)" : "hit gathering (grid walk)");
  if (gathered && (camera || n_batch > 0 || gathered->ws.last_hit_rays != n_rays))
    throw Error(SPH_HOA_E_INTERNAL, "shared gathering needs the same arbitrary rays");
  ws.collect_timing();
  ws.tuner.collect();
  ws.render_stats_pending = false;
  ws.stats = sph_hoa_stats{};
  ws.stats.n_rays = n_rays;
  ws.counters.ensure(256);
  unsigned long long* ctr = ws.counters.as<unsigned long long>();
  uint32_t* flags = reinterpret_cast<uint32_t*>(ctr + 16);
  unsigned int* queue = reinterpret_cast<unsigned int*>(ctr + 17);
  unsigned long long* max_hits = ctr + 18;
  hip_check(hipMemsetAsync(ws.counters.p, 0, 256, st), "memset");
  if (n_rays == 0) return;
  ws.rays_o.ensure(sizeof(double) * 3 * n_rays);
  ws.rays_v.ensure(sizeof(double) * 3 * n_rays);
  double t_min = 0.0, t_max = 0.0;
  const float* ray_tr = nullptr;
  const int n_cams = (n_batch > 0) ? n_batch : (camera ? 1 : 0);
  const sph_hoa_camera* cam_list = (n_batch > 0) ? batch : cam;
  CamDev* cdev = nullptr;
  int64_t *ray_base = nullptr, *tile_base = nullptr;
  int64_t n_tiles = 0;
  if (n_cams > 0) {
    // cameras (one, or a batch rendered together): frames, first ray and first screen tile of each
    std::vector<CamDev> cd((size_t)n_cams);
    std::vector<int64_t> rb((size_t)n_cams + 1, 0), tb((size_t)n_cams + 1, 0);
    for (int c = 0; c < n_cams; ++c) {
      const sph_hoa_camera& sc = cam_list[c];
      cd[c] = make_cam(&sc);
      rb[c + 1] = rb[c] + (int64_t)sc.width * sc.height;
      tb[c + 1] = tb[c] + (int64_t)((sc.width + kTile - 1) / kTile) * ((sc.height + kTile - 1) / kTile);
    }
    n_tiles = tb[n_cams];
    ws.cams_dev.ensure(sizeof(CamDev) * n_cams + sizeof(int64_t) * 2 * (n_cams + 1));
    cdev = ws.cams_dev.as<CamDev>();
    ray_base = reinterpret_cast<int64_t*>(cdev + n_cams);
    tile_base = ray_base + (n_cams + 1);
    hip_check(hipMemcpyAsync(cdev, cd.data(), sizeof(CamDev) * n_cams, hipMemcpyHostToDevice, st), "copy");
    hip_check(hipMemcpyAsync(ray_base, rb.data(), sizeof(int64_t) * (n_cams + 1), hipMemcpyHostToDevice, st), "copy");
    hip_check(hipMemcpyAsync(tile_base, tb.data(), sizeof(int64_t) * (n_cams + 1), hipMemcpyHostToDevice, st), "copy");
    ws.ray_tr.ensure(sizeof(float) * 2 * n_rays);
    k_camera_rays_batch<<<blocks_for(n_rays, 256), 256, 0, st>>>(cdev, ray_base, n_cams, n_rays, ws.rays_o.as<double>(),
                                                                 ws.rays_v.as<double>(), ws.ray_tr.as<float>());
    ray_tr = ws.ray_tr.as<float>();
    t_min = (double)cam_list[0].t_min;
    t_max = (double)cam_list[0].t_max;
    // the staged host vectors must outlive the copies
    hip_check(hipStreamSynchronize(st), "sync");
  } else {
    k_widen_rays<<<blocks_for(n_rays, 256), 256, 0, st>>>(rays->origin, rays->dir, n_rays, ws.rays_o.as<double>(),
                                                          ws.rays_v.as<double>(), flags);
    t_min = (double)rays->t_min;
    t_max = (double)rays->t_max;
  }
  hip_check(hipGetLastError(), "ray launch");
  // hit counts (another index's, when the gathering is shared)
  ws.hit_count.ensure(sizeof(int64_t) * (n_rays + 1));
  ws.hit_off.ensure(sizeof(int64_t) * (n_rays + 1));
  int64_t* hit_count = gathered ? gathered->ws.hit_count.as<int64_t>() : ws.hit_count.as<int64_t>();
  int64_t* hit_off = gathered ? gathered->ws.hit_off.as<int64_t>() : ws.hit_off.as<int64_t>();
  GatherArgs G{};
  G.o = ws.rays_o.as<double>();
  G.v = ws.rays_v.as<double>();
  G.n_rays = n_rays;
  G.t_min = t_min;
  G.t_max = t_max;
  G.pos4 = ix.pos4.as<float4>();
  G.cbeg = ix.cell_begin.as<uint32_t>();
  G.cend = ix.cell_end.as<uint32_t>();
  G.g = ix.grid;
  G.count = ws.hit_count.as<int64_t>();
  G.max_hits = max_hits;
  G.flags = flags;
  G.tr = ray_tr;
  const unsigned gblocks = (unsigned)((n_rays + 3) / 4);
  BinArgs B{};
  TileHitArgs TH{};
  const int64_t n_pairs_bin = ix.n * (int64_t)n_cams;
  int64_t n_slots = 0;  // arbitrary rays: per-ray hit slots of the single-pass gathering
  if (n_cams > 0) {
    // bin particles into screen tiles, then count hits per pixel ray from the tile lists
    B.pos4 = ix.pos4.as<float4>();
    B.n = ix.n;
    B.cams = cdev;
    B.tile_base = tile_base;
    B.n_cams = n_cams;
    ws.tile_count.ensure(sizeof(unsigned int) * (n_tiles + 1) * 2);
    ws.tile_off.ensure(sizeof(int64_t) * (n_tiles + 1) * 2);
    unsigned int* tcount = ws.tile_count.as<unsigned int>();
    unsigned int* tcur = tcount + (n_tiles + 1);
    int64_t* tcnt64 = ws.tile_off.as<int64_t>() + (n_tiles + 1);
    B.tile_count = tcount;
    B.tile_cursor = tcur;
    B.tile_off = ws.tile_off.as<int64_t>();
    if (ws.timing) hip_check(hipEventRecord(ws.ev[0], st), "event");
    hip_check(hipMemsetAsync(tcount, 0, sizeof(unsigned int) * (n_tiles + 1) * 2, st), "memset");
    k_bin<false><<<blocks_for(n_pairs_bin, 256), 256, 0, st>>>(B);
    k_u32_to_i64_n<<<blocks_for(n_tiles, 256), 256, 0, st>>>(tcount, tcnt64, n_tiles);
    device_exclusive_scan_i64(tcnt64, ws.tile_off.as<int64_t>(), n_tiles, ws.scan_tmp, st);
    k_set_last<<<1, 1, 0, st>>>(ws.tile_off.as<int64_t>(), tcnt64, n_tiles);
    int64_t n_items = 0;
    hip_check(hipMemcpyAsync(&n_items, ws.tile_off.as<int64_t>() + n_tiles, 8, hipMemcpyDeviceToHost, st), "copy");
    hip_check(hipStreamSynchronize(st), "sync");
    ws.tile_items.ensure(sizeof(uint32_t) * std::max<int64_t>(1, n_items));
    ws.tile_masks.ensure(sizeof(unsigned long long) * std::max<int64_t>(1, n_items));
    B.items = ws.tile_items.as<uint32_t>();
    k_bin<true><<<blocks_for(n_pairs_bin, 256), 256, 0, st>>>(B);
    TH.o = G.o;
    TH.v = G.v;
    TH.cams = cdev;
    TH.tile_base = tile_base;
    TH.ray_base = ray_base;
    TH.n_cams = n_cams;
    TH.pos4 = B.pos4;
    TH.tile_off = B.tile_off;
    TH.items = B.items;
    TH.masks = ws.tile_masks.as<unsigned long long>();
    {
      // tiles with the longest candidate lists first, so that they do not finish last
      ws.order_keys.ensure(sizeof(uint64_t) * 2 * n_tiles);
      uint64_t* k0 = ws.order_keys.as<uint64_t>();
      uint64_t* k1 = k0 + n_tiles;
      k_order_keys<<<blocks_for(n_tiles, 256), 256, 0, st>>>(tcnt64, n_tiles, k0);
      const bool alt = device_sort_u64(k0, k1, n_tiles, 64, ws.sort_hist, ws.sort_offs, ws.scan_tmp, st);
      ws.tile_order.ensure(sizeof(uint32_t) * n_tiles);
      k_low32<<<blocks_for(n_tiles, 256), 256, 0, st>>>(alt ? k1 : k0, n_tiles, ws.tile_order.as<uint32_t>());
      TH.order = ws.tile_order.as<uint32_t>();
    }
    TH.count = G.count;
    TH.max_hits = max_hits;
    k_tile_hits<false><<<(unsigned)n_tiles, 64, 0, st>>>(TH);
    if (ws.timing) hip_check(hipEventRecord(ws.ev[1], st), "event");
  } else if (gathered) {
    // the hit lists of the other index's call on these rays: no gathering (zero gathering time)
    if (ws.timing) {
      hip_check(hipEventRecord(ws.ev[0], st), "event");
      hip_check(hipEventRecord(ws.ev[1], st), "event");
    }
  } else {
    // Single pass when it fits: the counting walk also stores each ray's first n_slots hits in
    // per-ray slots, sized from the previous call's longest ray; the filling walk then runs only
    // if some ray has more hits than slots.
    int64_t want = ws.last_max_hits > 0 ? ws.last_max_hits : 256;
    n_slots = 16;
    while (n_slots < want) n_slots <<= 1;
    if (const char* f = std::getenv("SPH_HOA_GATHER_SLOTS")) n_slots = std::max<int64_t>(0, std::atoll(f));  // test hook
    if (n_slots > 0 && n_rays * n_slots > ((int64_t)1 << 30)) n_slots = 0;  // over 4 GiB: two walks
    if (n_slots > 0) {
      ws.hit_slots.ensure(sizeof(uint32_t) * n_rays * n_slots);
      G.slots = ws.hit_slots.as<uint32_t>();
      G.n_slots = n_slots;
    }
    if (ws.timing) hip_check(hipEventRecord(ws.ev[0], st), "event");
    k_gather<false><<<gblocks, kGatherThreads, 0, st>>>(G);
    if (ws.timing) hip_check(hipEventRecord(ws.ev[1], st), "event");
  }
  hip_check(hipGetLastError(), "gather launch");
  if (!gathered) {
    device_exclusive_scan_i64(hit_count, hit_off, n_rays, ws.scan_tmp, st);
    k_set_last<<<1, 1, 0, st>>>(hit_off, hit_count, n_rays);
  }
  int64_t total_pairs = 0;
  unsigned long long mh = 0;
  uint32_t fl = 0;
  hip_check(hipMemcpyAsync(&total_pairs, hit_off + n_rays, 8, hipMemcpyDeviceToHost, st), "copy");
  if (!gathered) hip_check(hipMemcpyAsync(&mh, max_hits, 8, hipMemcpyDeviceToHost, st), "copy");
  hip_check(hipMemcpyAsync(&fl, flags, 4, hipMemcpyDeviceToHost, st), "copy");
  hip_check(hipStreamSynchronize(st), "sync");
  if (gathered) mh = (unsigned long long)gathered->ws.last_hit_max;
  if (fl & kFlagBadInput) throw Error(SPH_HOA_E_INVALID_ARG, "ray origin/direction not finite or direction not unit");
  if (fl & kFlagWindow) throw Error(SPH_HOA_E_INTERNAL, "grid enumeration window exceeded");
  ws.stats.n_pairs = total_pairs;
  ws.stats.max_hits = (int64_t)mh;
  ws.stats.n_knots = total_pairs * (K + 1);
  // the per-ray sort ranks a wave's keys in 16-bit fields: at most 1023 keys per thread
  if ((int64_t)mh * (K + 1) > (int64_t)1023 * kFieldThreadsMin)
    throw Error(SPH_HOA_E_UNSUPPORTED, "more than 1023 * 256 knots on one ray");
  if (n_cams == 0) ws.last_max_hits = (int64_t)mh;
  const bool single_pass = gathered ? gathered->ws.last_hit_slots > 0 : (n_slots > 0 && (int64_t)mh <= n_slots);
  const uint32_t* hit_lists = nullptr;
  if (gathered) {
    hit_lists = single_pass ? gathered->ws.hit_slots.as<uint32_t>() : gathered->ws.hits.as<uint32_t>();
    n_slots = gathered->ws.last_hit_slots;
  } else if (single_pass) {
    hit_lists = ws.hit_slots.as<uint32_t>();
  } else {
    ws.hits.ensure(sizeof(uint32_t) * std::max<int64_t>(1, total_pairs));
    hit_lists = ws.hits.as<uint32_t>();
  }
  G.off = hit_off;
  G.hits = ws.hits.as<uint32_t>();
  G.slots = nullptr;
  if (ws.timing) hip_check(hipEventRecord(ws.ev[2], st), "event");
  if (n_cams > 0) {
    TH.off = G.off;
    TH.hits = G.hits;
    k_tile_hits<true><<<(unsigned)n_tiles, 64, 0, st>>>(TH);
  } else if (!single_pass && !gathered) {
    k_gather<true><<<gblocks, kGatherThreads, 0, st>>>(G);
  }
  const int64_t hit_slots = single_pass ? n_slots : 0;
  // the hit lists this index can share with the next call: its own, or none (its buffers may have
  // been resized) when it used another index's
  if (n_cams > 0 || (gathered && gathered != &ix)) {
    ws.last_hit_rays = -1;
  } else if (!gathered) {
    ws.last_hit_slots = hit_slots;
    ws.last_hit_rays = n_rays;
    ws.last_hit_max = (int64_t)mh;
  }
  if (ws.timing) hip_check(hipEventRecord(ws.ev[3], st), "event");
  hip_check(hipGetLastError(), "gather launch");
  if (out.hits) {
    HitsOut* ho = out.hits;
    ho->n_pairs = total_pairs;
    if (total_pairs > ho->capacity) throw Error(SPH_HOA_E_OUT_OF_MEMORY, "hit capacity too small");
    hip_check(hipMemcpyAsync(ho->offsets, hit_off, sizeof(int64_t) * (n_rays + 1), hipMemcpyDeviceToDevice, st),
              "copy");
    k_export_hits<<<(unsigned)std::min<int64_t>(n_rays, 1 << 20), 64, 0, st>>>(
        hit_off, hit_lists, hit_slots, n_rays, ix.orig.as<int32_t>(), ho->ids);
    hip_check(hipGetLastError(), "export launch");
    hip_check(hipStreamSynchronize(st), "sync");
    return;
  }
  if (out.flt) {
    // float accumulation variant: same hits, its own sweep
    if (ix.trans_axis >= 0) throw Error(SPH_HOA_E_UNSUPPORTED, "the float variant has no transverse fields");
    sph_hoa_float_field* ff = out.flt;
    const int64_t need = float_field_capacity(total_pairs, n_rays, K, out.n_reinit);
    ff->n_slots = need;
    ff->n_pairs = total_pairs;
    if (need > ff->capacity) throw Error(SPH_HOA_E_OUT_OF_MEMORY, "float field capacity too small");
    FloatArgs F{};
    F.o = G.o;
    F.v = G.v;
    F.n_rays = n_rays;
    F.t_min = t_min;
    F.t_max = t_max;
    F.hit_off = hit_off;
    F.hits = hit_lists;
    F.hit_slots = hit_slots;
    F.pos4 = ix.pos4.as<float4>();
    F.val = ix.val.as<float>();
    F.orig = ix.orig.as<int32_t>();
    F.theta = ix.lut_theta.as<double>();
    F.shat = ix.lut_shat.as<double>();
    F.smid = ix.lut_smid.as<double>();
    F.n_lut = ix.n_lut;
    F.K = K;
    F.P = P;
    F.even_k = (K % 2 == 0) ? 1 : 0;
    F.D = D;
    F.n_reinit = out.n_reinit;
    F.out_cnt = ff->ray_counts;
    F.t0 = ff->t_start;
    F.t1 = ff->t_end;
    F.coef = ff->coef;
    F.flags = flags;
    launch_float_field(F, (int64_t)mh, ix.float_scratch, ff->ray_offsets, st);
    uint32_t fl2 = 0;
    hip_check(hipMemcpyAsync(&fl2, flags, 4, hipMemcpyDeviceToHost, st), "copy");
    hip_check(hipStreamSynchronize(st), "sync");
    if (fl2 & kFlagCapacity) throw Error(SPH_HOA_E_INTERNAL, "float field wrote past its slots");
    return;
  }
  gather_range.reset();
  TraceRange field_range(out.rgba ? "field kernel (render)" : "field kernel (fields)");
  // ---- field kernel
  FieldArgs A{};
  A.o = G.o;
  A.v = G.v;
  A.n_rays = n_rays;
  A.t_min = t_min;
  A.t_max = t_max;
  A.tr = ray_tr;
  A.order = nullptr;
  if (n_cams != 1) {
    // arbitrary rays and batches can be heavy-tailed: process the longest rays first so that the
    // persistent work-groups finish together
    ws.order_keys.ensure(sizeof(uint64_t) * 2 * n_rays);
    uint64_t* k0 = ws.order_keys.as<uint64_t>();
    uint64_t* k1 = k0 + n_rays;
    k_order_keys<<<blocks_for(n_rays, 256), 256, 0, st>>>(hit_count, n_rays, k0);
    const bool alt = device_sort_u64(k0, k1, n_rays, 64, ws.sort_hist, ws.sort_offs, ws.scan_tmp, st);
    ws.order.ensure(sizeof(uint32_t) * n_rays);
    k_low32<<<blocks_for(n_rays, 256), 256, 0, st>>>(alt ? k1 : k0, n_rays, ws.order.as<uint32_t>());
    A.order = ws.order.as<uint32_t>();
  }
  A.hit_count = hit_count;
  A.hit_off = hit_off;
  A.hits = hit_lists;
  A.hit_slots = hit_slots;
  A.pos4 = ix.pos4.as<float4>();
  A.val = ix.val.as<float>();
  A.orig = ix.orig.as<int32_t>();
  // the table in its storage format: narrow copies when the index stores it narrow
  A.tab_fmt = ix.lut_fmt;
  A.trans_axis = ix.trans_axis;
  A.theta = ix.lut_fmt ? ix.lut_theta_n.p : ix.lut_theta.p;
  A.shat = ix.lut_fmt ? ix.lut_shat_n.p : ix.lut_shat.p;
  A.mc = MethodConsts{K, D, P, (K % 2 == 0) ? 1 : 0, ix.n_lut, (int)ix.kernel, ix.tau, ix.sigma, kSupport, ix.merge_tol};
  A.mt = make_merge_tables(D);
  A.queue = queue;
  A.flags = flags;
  A.counters = ctr;
  const int64_t max_knots = std::max<int64_t>(1, (int64_t)mh * (K + 1));
  A.max_knots = max_knots;
  // Work-groups per CU, 1 to 4: more ray work-groups per CU (one wave per SIMD each) hide more of
  // the latency of the dependent integer and float64 chains, fewer give each ray more LDS (long
  // rays keep more of their layout on chip).  Chosen per workload signature by measuring each
  // (FieldTuner); a ray's layout gets 1 / wgs of the CU's LDS less the static part, sized down to
  // the frame's longest ray.
  const int nj = jump_values_per_hit(P, (K % 2 == 0) ? 1 : 0, D);
  A.nj = nj;
  const int64_t mh1 = std::max<int64_t>(1, (int64_t)mh);
  const bool render_mode = (out.rgba != nullptr);
  const FieldTuner::Key tkey = FieldTuner::key_of(D, render_mode, total_pairs, n_rays, (int64_t)mh);
  // (the static-scratch entry point takes the tuner's choice without timing anything)
  int cfg = ws.no_alloc ? ws.tuner.chosen(tkey) : ws.tuner.choose(tkey);
  {
    // test hooks: a given number of work-groups per CU and of threads per work-group (the nearest
    // valid configuration)
    int w = field_cfg_wgs(cfg), t = field_cfg_threads(cfg);
    if (const char* f = std::getenv("SPH_HOA_FIELD_WGS")) w = std::min(4, std::max(1, std::atoi(f)));
    if (const char* f = std::getenv("SPH_HOA_FIELD_THREADS")) t = std::atoi(f) >= 512 ? 512 : 256;
    const int base = (t == 512 ? 4 : 0);
    if (!field_cfg_valid(D, render_mode, base + 1)) t = (t == 512 ? 256 : 512);  // the other thread count
    const int b = (t == 512 ? 4 : 0);
    if (t == 512) w = std::min(w, 2);
    while (w > 1 && !field_cfg_valid(D, render_mode, b + w)) --w;
    cfg = b + w;
  }
  const int wgs = field_cfg_wgs(cfg);
  const size_t lds_static = static_lds(D, field_cfg_threads(cfg));
  const int64_t lds_budget = kLdsPerCu / wgs - (int64_t)lds_static - 512;
  int64_t lds = std::min<int64_t>(lds_budget, ray_store_bytes(mh1, max_knots, nj, true));
  // test hook: a smaller LDS capacity (in hits) sends more rays down the device-memory paths
  if (const char* cap = std::getenv("SPH_HOA_MAX_LDS_HITS")) {
    const int64_t ch = std::max<int64_t>(1, std::atoll(cap));
    lds = std::min<int64_t>(lds, ray_store_bytes(ch, ch * (K + 1), nj, true));
  }
  A.lds_bytes = lds;
  hipDeviceProp_t prop;
  int dev = 0;
  hip_check(hipGetDevice(&dev), "device");
  hip_check(hipGetDeviceProperties(&prop, dev), "props");
  const int per_cu = (int)std::max<int64_t>(1, std::min<int64_t>(wgs, kLdsPerCu / (lds + (int64_t)lds_static + 512)));
  int grid = (int)std::min<int64_t>((int64_t)prop.multiProcessorCount * per_cu, n_rays);
  const int max_tier = ray_tier(mh1, max_knots, nj, lds);
  A.slab_jmp = align8((int64_t)node_bytes(D) * ((max_knots + kChunk - 1) / kChunk) * kChunk);
  A.slab_scratch = A.slab_jmp + (max_tier >= 1 ? align8(8 * (int64_t)nj * mh1) : 0);
  A.slab_store = A.slab_scratch + (max_tier >= 2 ? align8(8 * kpad_size(max_knots)) : 0);
  A.slab_stride = A.slab_store + (max_tier >= 3 ? align8(ray_store_bytes(mh1, max_knots, nj, true)) : 0) + 64;
  if (ws.slab.arena) {
    // fixed scratch: fewer persistent work-groups when their slabs do not all fit (same results)
    const int64_t fit = (int64_t)(ws.slab.room() / (size_t)A.slab_stride);
    if (fit < 1) throw Error(SPH_HOA_E_OUT_OF_MEMORY, "the longest ray needs more static scratch memory than is left");
    grid = (int)std::min<int64_t>(grid, fit);
  }
  ws.slab.ensure((size_t)A.slab_stride * grid);
  // Time slices: a workspace that shares the device with others (render server lanes) launches the
  // field kernel several times, each work-group taking a bounded share of the rays per launch, so
  // that the field work of batches on other streams starts within about one slice instead of
  // waiting for this batch's whole field kernel.  The last launch takes what rounding left over;
  // launches that find the queue drained end at once.
  int launches = 1;
  A.rays_per_wg = 0;
  int slices = ws.time_slices;
  if (const char* f = std::getenv("SPH_HOA_TIME_SLICES")) slices = std::max(1, std::atoi(f));  // test hook
  if (slices > 1 && n_rays > (int64_t)grid * slices) {
    A.rays_per_wg = (int)std::max<int64_t>(1, n_rays / ((int64_t)grid * slices));
    launches = (int)((n_rays + (int64_t)grid * A.rays_per_wg - 1) / ((int64_t)grid * A.rays_per_wg));
  }
  A.slab = ws.slab.as<char>();
  if (render_mode) {
    A.tf = out.tf->rgba;
    A.tf_n = out.tf->n;
    A.tf_vmin = out.tf->v_min;
    A.tf_vmax = out.tf->v_max;
    A.tf_step = (double)out.tf->step;
    A.rgba = out.rgba;
    if (ws.timing) hip_check(hipEventRecord(ws.ev[4], st), "event");
    if (!ws.no_alloc) ws.tuner.begin(tkey, cfg, total_pairs, st);
    for (int l = 0; l < launches; ++l) dispatch_field<true>(D, cfg, A, grid, (size_t)lds, st);
    if (!ws.no_alloc) ws.tuner.end(st);
    ws.render_stats_pending = true;
    if (ws.timing) {
      hip_check(hipEventRecord(ws.ev[5], st), "event");
      ws.timing_pending = true;
    }
  } else {
    sph_hoa_field* f = out.field;
    A.out_cap = f->capacity;
    ws.out_stage.ensure(std::max<size_t>(16, (size_t)f->capacity * sizeof(float) * (D + 3)));
    A.st_t0 = ws.out_stage.as<float>();
    A.st_t1 = A.st_t0 + f->capacity;
    A.st_coef = A.st_t1 + f->capacity;
    ws.ray_meta.ensure(sizeof(int64_t) * (4 * n_rays + 2));
    A.ray_out = ws.ray_meta.as<int64_t>();
    A.ray_ex = A.ray_out + 2 * n_rays;
    A.ray_peak = f->ray_peak;
    A.exact = out.exact ? 1 : 0;
    DevBuf knot_off;
    if (out.exact) {
      A.exact_cap = f->exact_capacity;
      ws.exact_stage.ensure(std::max<size_t>(16, (size_t)f->exact_capacity * sizeof(int64_t) * (D + 3)));
      A.ex_t = ws.exact_stage.as<int64_t>();
      A.ex_end = A.ex_t + f->exact_capacity;
      A.ex_coef = A.ex_end + f->exact_capacity;
      knot_off.ensure(sizeof(int64_t) * (n_rays + 1));
      k_scale_i64<<<blocks_for(n_rays + 1, 256), 256, 0, st>>>(hit_off, knot_off.as<int64_t>(),
                                                               n_rays + 1, K + 1);
      A.knot_off = knot_off.as<int64_t>();
      A.knot_cap = f->knot_capacity;
      A.kn_t = f->knot_t;
      A.kn_pid = f->knot_pid;
      A.kn_kidx = f->knot_kidx;
      if (f->knot_offsets)
        hip_check(hipMemcpyAsync(f->knot_offsets, knot_off.p, sizeof(int64_t) * (n_rays + 1), hipMemcpyDeviceToDevice, st),
                  "copy");
    }
    if (ws.timing) hip_check(hipEventRecord(ws.ev[4], st), "event");
    if (!ws.no_alloc) ws.tuner.begin(tkey, cfg, total_pairs, st);
    for (int l = 0; l < launches; ++l) dispatch_field<false>(D, cfg, A, grid, (size_t)lds, st);
    if (!ws.no_alloc) ws.tuner.end(st);
    if (ws.timing) {
      hip_check(hipEventRecord(ws.ev[5], st), "event");
      ws.timing_pending = true;
    }
    // counts -> final offsets, then reorder staged pieces by ray
    DevBuf cnt;
    cnt.ensure(sizeof(int64_t) * (n_rays + 1));
    k_ray_counts<<<blocks_for(n_rays, 256), 256, 0, st>>>(A.ray_out, n_rays, cnt.as<int64_t>());
    device_exclusive_scan_i64(cnt.as<int64_t>(), f->ray_offsets, n_rays, ws.scan_tmp, st);
    k_set_last<<<1, 1, 0, st>>>(f->ray_offsets, cnt.as<int64_t>(), n_rays);
    unsigned long long c4[6];
    hip_check(hipMemcpyAsync(c4, ctr, sizeof(c4), hipMemcpyDeviceToHost, st), "copy");
    hip_check(hipMemcpyAsync(&fl, flags, 4, hipMemcpyDeviceToHost, st), "copy");
    hip_check(hipStreamSynchronize(st), "sync");
    f->n_pieces = (int64_t)c4[0];
    f->n_exact_pieces = (int64_t)c4[2];
    f->n_pairs = total_pairs;
    f->n_knots = total_pairs * (K + 1);
    ws.stats.n_pieces = (int64_t)c4[0];
    ws.stats.rays_global = (int64_t)c4[3];
    ws.stats.rays_jumps_device = (int64_t)c4[4];
    ws.stats.rays_scratch_device = (int64_t)c4[5];
    if (fl & kFlagPosRange)
      throw Error(SPH_HOA_E_OVERFLOW, "a ray's knots span 2^32 length quanta or more, or a knot offset q h / tau "
                                      "reached 2^31");
    if (fl & kFlagCoefRange) throw Error(SPH_HOA_E_OVERFLOW, "a quantized coefficient left the int64 range");
    if (fl & kFlagTail) throw Error(SPH_HOA_E_INTERNAL, "a ray's knots did not cancel exactly");
    bool short_cap = f->n_pieces > f->capacity;
    if (out.exact) short_cap = short_cap || f->n_exact_pieces > f->exact_capacity || f->n_knots > f->knot_capacity;
    if (short_cap) throw Error(SPH_HOA_E_OUT_OF_MEMORY, "output capacity too small");
    k_copy_pieces<<<(unsigned)n_rays, 64, 0, st>>>(A.ray_out, f->ray_offsets, n_rays, D + 1, A.st_t0, A.st_t1,
                                                   A.st_coef, f->t_start, f->t_end, f->coef);
    if (out.exact) {
      k_ray_counts<<<blocks_for(n_rays, 256), 256, 0, st>>>(A.ray_ex, n_rays, cnt.as<int64_t>());
      device_exclusive_scan_i64(cnt.as<int64_t>(), f->exact_offsets, n_rays, ws.scan_tmp, st);
      k_set_last<<<1, 1, 0, st>>>(f->exact_offsets, cnt.as<int64_t>(), n_rays);
      k_copy_exact<<<(unsigned)n_rays, 64, 0, st>>>(A.ray_ex, f->exact_offsets, n_rays, D + 1, A.ex_t, A.ex_end,
                                                    A.ex_coef, f->exact_t, f->exact_end, f->exact_coef);
    }
    hip_check(hipGetLastError(), "copy launch");
    hip_check(hipStreamSynchronize(st), "sync");
    return;
  }
  if (!workspace) ix.last_stream = st;  // lanes of the render server keep their own streams
}

}  // namespace sph
