// Integer bit length of the accumulation (Sec. 5.1, performance implications of the integer
// representation).
//
// The paper weighs its integer update rule (Eq. accumulation-rule) at 32-bit integers against
// software-emulated 64, 96 and 128 bits, which it puts at roughly 9, 24 and 45 times the cost of
// a 32-bit operation.  This kernel applies the rule - a Taylor shift of the D + 1 localized
// coefficients by the distance to the next knot, D (D + 1) / 2 multiply-adds of a W-bit
// coefficient by the 32-bit distance, then the knot's jump added - in wrap-around W-bit
// arithmetic as the compiler lowers it, so that the cost of each width can be measured on gfx950
// on the same work (the compiler may rewrite the shift, e.g. merge repeated products, alike for
// every width).  The distance is a 32-bit factor because on one ray the distance between two
// knots, in length quanta, fits 32 bits (the field kernel makes the same W x 32 products with
// W = 64).
//
// Each thread runs its own accumulation over a cycle of four knots held in registers (table
// entries (g + e) mod n_table for e = 0..3, g the thread's index), so that the timed loop is the
// rule's arithmetic alone: knot s of thread g is entry (g + s mod 4) mod n_table.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "impl.h"

namespace sph {
namespace {

constexpr int kCycle = 4;

// W-bit unsigned integers with wrap-around arithmetic, lowered by the compiler into 32-bit
// operations (gfx950 has no wider integer multiply than 32 x 32 -> 64 bits): the software
// emulation the cost study is about.
template <int L>
using Wide = unsigned _BitInt(32 * L);

// The jumps of the four-knot cycle are loop invariants, so without a barrier the compiler turns
// the top coefficient (which only accumulates jumps) into an induction variable and replaces its
// products by additions - work the rule cannot skip when jumps come from memory.  The empty asm
// on each 32-bit limb makes the state opaque at every knot and emits no instruction.
template <int L>
__device__ __forceinline__ void opaque(Wide<L>& x) {
  uint32_t limb[L];
#pragma unroll
  for (int i = 0; i < L; ++i) {
    limb[i] = (uint32_t)(x >> (32 * i));
    asm("" : "+v"(limb[i]));
  }
  Wide<L> r = 0;
#pragma unroll
  for (int i = 0; i < L; ++i) r |= (Wide<L>)limb[i] << (32 * i);
  x = r;
}

// One knot of the rule: Taylor shift of the localized coefficients by the 32-bit distance d
// (in place, from the top coefficient down), then the knot's jump added.
template <int L, int D>
__device__ __forceinline__ void knot_step(Wide<L> (&a)[D + 1], uint32_t d, const Wide<L> (&jump)[D + 1]) {
#pragma unroll
  for (int k = 0; k <= D; ++k) opaque<L>(a[k]);
  const Wide<L> dw = (Wide<L>)d;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = D - 1; j >= i; --j) a[j] += a[j + 1] * dw;
#pragma unroll
  for (int k = 0; k <= D; ++k) a[k] += jump[k];
}

template <int L, int D>
__global__ void __launch_bounds__(256) k_accumulate_bits(const uint32_t* __restrict__ dist,
                                                        const uint32_t* __restrict__ jumps, int n_table, int cycles,
                                                        int64_t n_threads, uint32_t* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_threads) return;
  uint32_t dd[kCycle];
  Wide<L> jp[kCycle][D + 1];
#pragma unroll
  for (int e = 0; e < kCycle; ++e) {
    const int k = (int)((g + e) % n_table);
    dd[e] = dist[k];
#pragma unroll
    for (int d = 0; d <= D; ++d) {
      Wide<L> v = 0;
#pragma unroll
      for (int i = 0; i < L; ++i) v |= (Wide<L>)jumps[((int64_t)k * (D + 1) + d) * L + i] << (32 * i);
      jp[e][d] = v;
    }
  }
  Wide<L> a[D + 1];
#pragma unroll
  for (int d = 0; d <= D; ++d) a[d] = jp[0][d];  // first knot: the state is its jump
#pragma unroll
  for (int e = 1; e < kCycle; ++e) knot_step<L, D>(a, dd[e], jp[e]);
  for (int c = 1; c < cycles; ++c) {
#pragma unroll
    for (int e = 0; e < kCycle; ++e) knot_step<L, D>(a, dd[e], jp[e]);
  }
#pragma unroll
  for (int d = 0; d <= D; ++d)
#pragma unroll
    for (int i = 0; i < L; ++i) out[(g * (D + 1) + d) * L + i] = (uint32_t)(a[d] >> (32 * i));
}

template <int L, int D>
void launch_bits(const uint32_t* dist, const uint32_t* jumps, int n_table, int cycles, int64_t n_threads,
                 uint32_t* out, hipStream_t st) {
  const unsigned blocks = (unsigned)((n_threads + 255) / 256);
  k_accumulate_bits<L, D><<<blocks, 256, 0, st>>>(dist, jumps, n_table, cycles, n_threads, out);
}

template <int L>
void dispatch_degree(int D, const uint32_t* dist, const uint32_t* jumps, int n_table, int cycles, int64_t n_threads,
                     uint32_t* out, hipStream_t st) {
  switch (D) {
    case 1: launch_bits<L, 1>(dist, jumps, n_table, cycles, n_threads, out, st); break;
    case 2: launch_bits<L, 2>(dist, jumps, n_table, cycles, n_threads, out, st); break;
    case 3: launch_bits<L, 3>(dist, jumps, n_table, cycles, n_threads, out, st); break;
    case 4: launch_bits<L, 4>(dist, jumps, n_table, cycles, n_threads, out, st); break;
    case 5: launch_bits<L, 5>(dist, jumps, n_table, cycles, n_threads, out, st); break;
    default: launch_bits<L, 6>(dist, jumps, n_table, cycles, n_threads, out, st); break;
  }
}

}  // namespace

void accumulate_bits(int bits, int D, const uint32_t* dist, const uint32_t* jumps, int n_table, int64_t n_threads,
                     int steps, uint32_t* out_host, float* ms, hipStream_t st) {
  if (bits != 32 && bits != 64 && bits != 96 && bits != 128)
    throw Error(SPH_HOA_E_INVALID_ARG, "bits must be 32, 64, 96 or 128");
  if (D < 1 || D > kMaxD) throw Error(SPH_HOA_E_INVALID_ARG, "degree must be in 1..6");
  if (n_table < 1) throw Error(SPH_HOA_E_INVALID_ARG, "table length must be >= 1");
  if (n_threads < 1 || n_threads > (int64_t)1 << 26) throw Error(SPH_HOA_E_INVALID_ARG, "threads must be in 1..2^26");
  if (steps < kCycle || steps % kCycle != 0) throw Error(SPH_HOA_E_INVALID_ARG, "steps must be a positive multiple of 4");
  const int L = bits / 32;
  const size_t row = (size_t)(D + 1) * L;
  DevBuf d_dist, d_jump, d_out;
  d_dist.ensure(sizeof(uint32_t) * n_table);
  d_jump.ensure(sizeof(uint32_t) * (size_t)n_table * row);
  d_out.ensure(sizeof(uint32_t) * (size_t)n_threads * row);
  hip_check(hipMemcpyAsync(d_dist.p, dist, sizeof(uint32_t) * n_table, hipMemcpyHostToDevice, st), "copy");
  hip_check(hipMemcpyAsync(d_jump.p, jumps, sizeof(uint32_t) * (size_t)n_table * row, hipMemcpyHostToDevice, st),
            "copy");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hip_check(hipEventCreate(&e0), "event");
  hip_check(hipEventCreate(&e1), "event");
  float t = 0.f;
  try {
    hip_check(hipEventRecord(e0, st), "event");
    const uint32_t* a = d_dist.as<uint32_t>();
    const uint32_t* b = d_jump.as<uint32_t>();
    uint32_t* o = d_out.as<uint32_t>();
    const int cycles = steps / kCycle;
    switch (L) {
      case 1: dispatch_degree<1>(D, a, b, n_table, cycles, n_threads, o, st); break;
      case 2: dispatch_degree<2>(D, a, b, n_table, cycles, n_threads, o, st); break;
      case 3: dispatch_degree<3>(D, a, b, n_table, cycles, n_threads, o, st); break;
      default: dispatch_degree<4>(D, a, b, n_table, cycles, n_threads, o, st); break;
    }
    hip_check(hipGetLastError(), "launch");
    hip_check(hipEventRecord(e1, st), "event");
    hip_check(hipEventSynchronize(e1), "event sync");
    hip_check(hipEventElapsedTime(&t, e0, e1), "elapsed");
    if (out_host)
      hip_check(hipMemcpy(out_host, o, sizeof(uint32_t) * (size_t)n_threads * row, hipMemcpyDeviceToHost), "copy");
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ms) *ms = t;
}

}  // namespace sph
