// Float accumulation variant (Sec. 4.1): the update rule swept along each ray in float32, with
// optional reinitialization knots, as an A/B against the exact integer path.
//
// The paper explains why it quantizes: applying the update rule (Eq. accumulation-rule) to float
// coefficients from front to back lets rounding errors of the higher-order coefficients grow with
// the distance along the ray, so the field does not return to zero behind the particles
// ("sprinkling", Fig. 2a).  As a partial remedy it describes reinitialization knots at fixed
// positions on every ray: each particle adds to every reinitialization knot it covers its own
// localized coefficients there, and the sweep takes those coefficients at such a knot instead of
// the updated ones (Fig. 2b).  This file computes that float sweep for arbitrary rays, one ray per
// work-group, so that its error can be measured against the exact path.
//
// Per hit (same hit set, closest-point parameter, distance parameter and table entry as the exact
// path): with tc, zf and vf the float32 roundings of t_chi, zeta and the amplitude, the knots sit
// at tc -+ zf * theta_k (and tc for even K), and the jump of order d >= 1 at +theta_k is
// s-hat_kd * vf / zf^(3 + d) (each power formed by repeated multiplication by 1 / zf), at -theta_k
// the same times (-1)^(d + 1), at 0 the table's middle jump (even K).  Knots are ordered by
// (position, particle input index, kidx).  One thread sweeps them: the state is shifted to each
// knot position (the in-place Taylor shift, top coefficient down) and the jump added; a
// reinitialization knot at T takes effect after every knot at positions <= T.  The sweep emits one
// piece per gap between consecutive event positions, localized at its start, and a last piece
// from the final event to t_max holding what is left of the field behind the particles (zero in
// exact arithmetic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device.h"
#include "impl.h"

namespace sph {
namespace {

constexpr int kFloatThreads = 256;

__device__ __forceinline__ uint32_t float_order_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// per-work-group scratch, carved from one slab (all 8-byte aligned)
struct FloatScratch {
  uint64_t *hkey, *htmp;     // [cap_h] (orig << 32 | slot), sorted by orig
  uint32_t* rank_of_slot;    // [cap_h]
  uint32_t* slot_of_rank;    // [cap_h]
  uint64_t *kkey, *ktmp;     // [cap_k] (order bits << 32 | rank << 3 | kidx)
  float* kpos;               // [cap_k] knot positions, by knot id = slot * (K + 1) + slotk
  float* kcoef;              // [cap_k][D + 1] jumps
  float* loc;                // [cap_h][D + 1] localized coefficients at one reinitialization knot
  float* reinit;             // [n_reinit][D + 1]
};

__host__ __device__ inline int64_t float_scratch_bytes(int64_t cap_h, int K, int D, int n_reinit) {
  const int64_t cap_k = cap_h * (K + 1);
  auto a8 = [](int64_t b) { return (b + 7) & ~(int64_t)7; };
  return 16 * cap_h + a8(8 * cap_h) + 16 * cap_k + a8(4 * cap_k) + a8(4 * cap_k * (D + 1)) +
         a8(4 * cap_h * (D + 1)) + a8(4 * (int64_t)n_reinit * (D + 1));
}

__device__ inline FloatScratch carve_float(char* p, int64_t cap_h, int K, int D, int n_reinit) {
  const int64_t cap_k = cap_h * (K + 1);
  auto a8 = [](int64_t b) { return (b + 7) & ~(int64_t)7; };
  FloatScratch S;
  S.hkey = reinterpret_cast<uint64_t*>(p);
  S.htmp = S.hkey + cap_h;
  p += 16 * cap_h;
  S.rank_of_slot = reinterpret_cast<uint32_t*>(p);
  S.slot_of_rank = S.rank_of_slot + cap_h;
  p += a8(8 * cap_h);
  S.kkey = reinterpret_cast<uint64_t*>(p);
  S.ktmp = S.kkey + cap_k;
  p += 16 * cap_k;
  S.kpos = reinterpret_cast<float*>(p);
  p += a8(4 * cap_k);
  S.kcoef = reinterpret_cast<float*>(p);
  p += a8(4 * cap_k * (D + 1));
  S.loc = reinterpret_cast<float*>(p);
  p += a8(4 * cap_h * (D + 1));
  S.reinit = reinterpret_cast<float*>(p);
  return S;
}

template <int D>
__device__ __forceinline__ void shift_f(float* a, float delta) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = D - 1; j >= i; --j) a[j] = a[j] + a[j + 1] * delta;
}

// kidx of a particle's slotk-th knot (knots in increasing kidx; odd K has no middle knot)
__device__ __forceinline__ int kidx_of(int slotk, int P, int even_k) {
  return even_k ? slotk : (slotk < P ? slotk : slotk + 1);
}

template <int D>
__global__ void __launch_bounds__(kFloatThreads) k_float_field(FloatArgs F) {
  __shared__ uint32_t tab[32 * (kFloatThreads / 64)];
  const int tid = threadIdx.x;
  const int K = F.K, P = F.P, even_k = F.even_k, K1 = F.K + 1;
  FloatScratch S = carve_float(F.scratch + (int64_t)blockIdx.x * F.scratch_stride, F.cap_h, K, D, F.n_reinit);
  const float tmin_f = (float)F.t_min, tmax_f = (float)F.t_max;
  const float step_f = (tmax_f - tmin_f) / (float)(F.n_reinit + 1);
  for (int64_t r = blockIdx.x; r < F.n_rays; r += gridDim.x) {
    const int64_t hoff = F.hit_slots ? r * F.hit_slots : F.hit_off[r];
    const int nh = (int)(F.hit_off[r + 1] - F.hit_off[r]);
    const int nk = nh * K1;
    double o[3], v[3];
    for (int k = 0; k < 3; ++k) {
      o[k] = F.o[3 * r + k];
      v[k] = F.v[3 * r + k];
    }
    __syncthreads();  // the previous ray's sweep is done with the scratch
    // ---- knots and jumps of every hit, and the (input index, slot) keys for the ranks
    for (int s = tid; s < nh; s += kFloatThreads) {
      const uint32_t j = F.hits[hoff + s];
      const float4 p = F.pos4[j];
      const double dxx = (double)p.x - o[0], dxy = (double)p.y - o[1], dxz = (double)p.z - o[2];
      const double cx = dxy * v[2] - dxz * v[1];
      const double cy = dxz * v[0] - dxx * v[2];
      const double cz = dxx * v[1] - dxy * v[0];
      const double z = (double)p.w;
      const double lam2 = (cx * cx + cy * cy + cz * cz) / (z * z);
      const double tchi = dxx * v[0] + dxy * v[1] + dxz * v[2];
      int li = (int)floor(sqrt(lam2) * (double)F.n_lut / kSupport);
      li = li < 0 ? 0 : (li > F.n_lut - 1 ? F.n_lut - 1 : li);
      const float tc = (float)tchi, zf = p.w, vf = F.val[j];
      const float inv = 1.0f / zf;
      const float base = vf * inv * inv * inv;
      float sc[D + 1];
      sc[0] = base;
#pragma unroll
      for (int d = 1; d <= D; ++d) sc[d] = sc[d - 1] * inv;
      for (int slotk = 0; slotk < K1; ++slotk) {
        const int kidx = kidx_of(slotk, P, even_k);
        const int k = kidx - P;
        const int m = (k < 0 ? -k : k) - 1;  // table row of +-theta_|k| (m < 0: middle knot)
        float t = tc;
        if (m >= 0) {
          const float off = zf * (float)F.theta[(int64_t)li * P + m];
          t = (k < 0) ? tc - off : tc + off;
        }
        t = t + 0.0f;  // no negative zero in the ordering
        const int64_t q = (int64_t)s * K1 + slotk;
        S.kpos[q] = t;
        float* c = S.kcoef + q * (D + 1);
        c[0] = 0.0f;
#pragma unroll
        for (int d = 1; d <= D; ++d) {
          const double sh = (m >= 0) ? F.shat[((int64_t)li * P + m) * (D + 1) + d] : F.smid[(int64_t)li * (D + 1) + d];
          float x = (float)sh * sc[d];
          if (k < 0 && (d % 2 == 0)) x = -x;
          c[d] = x;
        }
      }
      S.hkey[s] = ((uint64_t)(uint32_t)F.orig[j] << 32) | (uint32_t)s;
    }
    __syncthreads();
    radix_sort_u64<kFloatThreads, false>(S.hkey, S.htmp, nh, 32, 32, tab, tid);
    for (int i = tid; i < nh; i += kFloatThreads) {
      const uint32_t s = (uint32_t)S.hkey[i];
      S.slot_of_rank[i] = s;
      S.rank_of_slot[s] = (uint32_t)i;
    }
    __syncthreads();
    for (int q = tid; q < nk; q += kFloatThreads) {
      const int s = q / K1, slotk = q % K1;
      S.kkey[q] = ((uint64_t)float_order_bits(S.kpos[q]) << 32) | ((uint64_t)S.rank_of_slot[s] << 3) |
                  (uint64_t)kidx_of(slotk, P, even_k);
    }
    __syncthreads();
    radix_sort_u64<kFloatThreads, false>(S.kkey, S.ktmp, nk, 0, 64, tab, tid);
    // ---- reinitialization knots: every covering particle's localized coefficients, summed in
    // increasing particle input index
    for (int sl = 0; sl < F.n_reinit; ++sl) {
      const float T = tmin_f + (float)(sl + 1) * step_f;
      for (int s = tid; s < nh; s += kFloatThreads) {
        float* L = S.loc + (int64_t)s * (D + 1);
        const float first = S.kpos[(int64_t)s * K1], last = S.kpos[(int64_t)s * K1 + K];
        float st[D + 1];
#pragma unroll
        for (int d = 0; d <= D; ++d) st[d] = 0.0f;
        if (first <= T && T < last) {
          float prev = first;
          for (int slotk = 0; slotk < K1; ++slotk) {
            const int64_t q = (int64_t)s * K1 + slotk;
            const float t = S.kpos[q];
            if (t > T) break;
            if (slotk > 0) shift_f<D>(st, t - prev);
#pragma unroll
            for (int d = 0; d <= D; ++d) st[d] = st[d] + S.kcoef[q * (D + 1) + d];
            prev = t;
          }
          shift_f<D>(st, T - prev);
        }
#pragma unroll
        for (int d = 0; d <= D; ++d) L[d] = st[d];
      }
      __syncthreads();
      if (tid == 0) {
        float acc[D + 1];
#pragma unroll
        for (int d = 0; d <= D; ++d) acc[d] = 0.0f;
        for (int i = 0; i < nh; ++i) {
          const float* L = S.loc + (int64_t)S.slot_of_rank[i] * (D + 1);
#pragma unroll
          for (int d = 0; d <= D; ++d) acc[d] = acc[d] + L[d];
        }
#pragma unroll
        for (int d = 0; d <= D; ++d) S.reinit[sl * (D + 1) + d] = acc[d];
      }
      __syncthreads();
    }
    // ---- the sweep
    if (tid == 0) {
      const int64_t base_out = F.out_off[r], cap = F.out_off[r + 1] - base_out;
      int64_t np = 0;
      auto emit = [&](float a, float b, const float* c) {
        if (np < cap) {
          const int64_t e = base_out + np;
          F.t0[e] = a;
          F.t1[e] = b;
#pragma unroll
          for (int d = 0; d <= D; ++d) F.coef[e * (D + 1) + d] = c[d];
        }
        ++np;
      };
      float st[D + 1];
#pragma unroll
      for (int d = 0; d <= D; ++d) st[d] = 0.0f;
      bool have = false;
      float prev = 0.0f;
      int sl = 0;
      auto reinit_upto = [&](float t, bool inclusive) {
        // reinitialization knots before t (all remaining ones when inclusive)
        while (sl < F.n_reinit) {
          const float T = tmin_f + (float)(sl + 1) * step_f;
          if (!inclusive && !(T < t)) break;
          if (have && T > prev) emit(prev, T, st);
#pragma unroll
          for (int d = 0; d <= D; ++d) st[d] = S.reinit[sl * (D + 1) + d];
          prev = T;
          have = true;
          ++sl;
        }
      };
      for (int i = 0; i < nk; ++i) {
        const uint64_t key = S.kkey[i];
        const uint32_t rank = (uint32_t)(key >> 3) & 0x1fffffffu;
        const int kidx = (int)(key & 7u);
        const int slotk = even_k ? kidx : (kidx < P ? kidx : kidx - 1);
        const int64_t q = (int64_t)S.slot_of_rank[rank] * K1 + slotk;
        const float t = S.kpos[q];
        reinit_upto(t, false);
        if (have && t > prev) emit(prev, t, st);
        if (have) shift_f<D>(st, t - prev);
#pragma unroll
        for (int d = 0; d <= D; ++d) st[d] = st[d] + S.kcoef[q * (D + 1) + d];
        prev = t;
        have = true;
      }
      reinit_upto(0.0f, true);
      if (have && prev < tmax_f) emit(prev, tmax_f, st);
      F.out_cnt[r] = np;
      if (np > cap) atomicOr(F.flags, kFlagCapacity);
    }
  }
}

__global__ void k_float_offsets(const int64_t* hit_off, int64_t n, int K1, int per_ray, int64_t* out_off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n) out_off[i] = hit_off[i] * K1 + i * per_ray;
}

}  // namespace

int64_t float_field_capacity(int64_t total_pairs, int64_t n_rays, int K, int n_reinit) {
  return total_pairs * (K + 1) + n_rays * (int64_t)(n_reinit + 2);
}

void launch_float_field(FloatArgs& F, int64_t max_hits, DevBuf& scratch, int64_t* out_off, hipStream_t st) {
  if (F.n_rays == 0) return;
  F.cap_h = std::max<int64_t>(1, max_hits);
  F.scratch_stride = float_scratch_bytes(F.cap_h, F.K, F.D, F.n_reinit);
  F.scratch_stride = (F.scratch_stride + 255) & ~(int64_t)255;
  // one ray per work-group at a time; the sweep is one thread's, so many work-groups per CU keep
  // the CUs busy.  Scratch per work-group scales with the longest ray: bounded to 4 GiB in total.
  const int64_t by_memory = std::max<int64_t>(1, ((int64_t)4 << 30) / F.scratch_stride);
  const int grid = (int)std::min<int64_t>(std::min<int64_t>(F.n_rays, 8192), by_memory);
  scratch.ensure((size_t)F.scratch_stride * grid);
  F.scratch = scratch.as<char>();
  k_float_offsets<<<(unsigned)((F.n_rays + 1 + 255) / 256), 256, 0, st>>>(F.hit_off, F.n_rays, F.K + 1,
                                                                           F.n_reinit + 2, out_off);
  F.out_off = out_off;
  switch (F.D) {
    case 1: k_float_field<1><<<grid, kFloatThreads, 0, st>>>(F); break;
    case 2: k_float_field<2><<<grid, kFloatThreads, 0, st>>>(F); break;
    case 3: k_float_field<3><<<grid, kFloatThreads, 0, st>>>(F); break;
    case 4: k_float_field<4><<<grid, kFloatThreads, 0, st>>>(F); break;
    case 5: k_float_field<5><<<grid, kFloatThreads, 0, st>>>(F); break;
    default: k_float_field<6><<<grid, kFloatThreads, 0, st>>>(F); break;
  }
  hip_check(hipGetLastError(), "float field launch");
}

}  // namespace sph
