// Projection of the table entries on the device (Sec. 3.1, 3.3, App. A.1/A.2): for every entry
// Lambda_i = (i + 1/2) q / n with its positive knots theta (from the knot optimisation of Sec. 3.4),
// the L2 projection of B_Lambda(t) = w(sqrt(Lambda^2 + t^2)) onto the even piecewise polynomials
// with those knots, returned as localized jump coefficients.  One wave per entry: the quadrature
// nodes are laid out in LDS, every lane forms entries of the normal equations G c = b (inner
// products over the nodes in node order, as the host builder sums them), and one lane solves the
// small system (|J| = floor(K D / 2) <= 18 unknowns) and converts the solution into jumps.
//
// The normal equations of an entry are a |J| x |J| Gram matrix over a few hundred nodes: about
// 1e5 float64 multiply-adds per entry, 4e8 for a 4096-entry table, done once per (kernel, K, D,
// table size).  Matrices this small would leave a matrix-core tile mostly empty, so the kernel
// uses plain float64 vector arithmetic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>
#include <vector>

#include "impl.h"
#include "lutmath.h"

namespace sph {
namespace {

constexpr int kLutMaxNodes = 1024;  // at most ~530 for tables of up to 65536 entries
constexpr int kLutMaxBasis = 18;

struct LutProjArgs {
  Kernel kernel;
  int K, D, P, n, nb;
  int bk[kLutMaxBasis], bd[kLutMaxBasis];
  double glx[kLutGL], glw[kLutGL];
  const double* theta;  // [n][P]
  double* shat;         // [n][P][D + 1]
  double* smid;         // [n][D + 1]
  double* err2;         // [n]
  uint32_t* status;     // bit 0: knots not positive increasing; bit 1: too many nodes; bit 2: singular
};

__global__ __launch_bounds__(64) void k_lut_project(LutProjArgs A) {
  __shared__ QuadPlan plan;
  __shared__ double nt[kLutMaxNodes], nw[kLutMaxNodes], nB[kLutMaxNodes];
  __shared__ double G[kLutMaxBasis * kLutMaxBasis], rhs[kLutMaxBasis];
  __shared__ double th[8];
  __shared__ int ok, M;
  const int e = blockIdx.x, lane = threadIdx.x;
  const int P = A.P, nb = A.nb, D = A.D;
  const double lam = (e + 0.5) * kSupport / A.n;
  if (lane == 0) {
    th[0] = 0.0;
    int valid = 1;
    for (int i = 0; i < P; ++i) {
      th[i + 1] = A.theta[(size_t)e * P + i];
      if (!(th[i + 1] > th[i])) valid = 0;
    }
    if (valid) {
      quad_plan(A.kernel, lam, th + 1, P, plan);
      M = plan.first[plan.nseg];
      if (M > kLutMaxNodes) {
        valid = 0;
        atomicOr(A.status, 2u);
      }
    } else {
      atomicOr(A.status, 1u);
    }
    ok = valid;
  }
  __syncthreads();
  if (!ok) {
    if (lane == 0) A.err2[e] = __builtin_inf();
    return;
  }
  const int m = M;
  for (int j = lane; j < m; j += 64) quad_node(A.kernel, plan, A.glx, A.glw, j, &nt[j], &nw[j], &nB[j]);
  __syncthreads();
  // entries of G (lower triangle, pair p -> (i, l), l <= i) and of b, each a sum over the nodes in
  // node order
  const int npairs = nb * (nb + 1) / 2;
  for (int p = lane; p < npairs + nb; p += 64) {
    if (p < npairs) {
      int i = 0;
      while ((i + 1) * (i + 2) / 2 <= p) ++i;
      const int l = p - i * (i + 1) / 2;
      const int ki = A.bk[i], di = A.bd[i], kl = A.bk[l], dl = A.bd[l];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += nw[j] * basis_val(th, ki, di, nt[j]) * basis_val(th, kl, dl, nt[j]);
      G[i * nb + l] = 2.0 * s;
      G[l * nb + i] = 2.0 * s;
    } else {
      const int i = p - npairs;
      const int ki = A.bk[i], di = A.bd[i];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += nw[j] * basis_val(th, ki, di, nt[j]) * nB[j];
      rhs[i] = 2.0 * s;
    }
  }
  __syncthreads();
  if (lane != 0) return;
  double c[kLutMaxBasis];
  for (int i = 0; i < nb; ++i) c[i] = rhs[i];
  if (!lut_chol_solve(G, c, nb)) {
    atomicOr(A.status, 4u);
    A.err2[e] = __builtin_inf();
    return;
  }
  double e2 = 0.0;
  for (int j = 0; j < m; ++j) {
    double S = 0.0;
    for (int i = 0; i < nb; ++i) S += c[i] * basis_val(th, A.bk[i], A.bd[i], nt[j]);
    const double R = nB[j] - S;
    e2 += nw[j] * R * R;
  }
  A.err2[e] = 2.0 * e2;
  lut_jumps(A.K, D, A.bk, A.bd, nb, th + 1, c, A.shat + (size_t)e * P * (D + 1), A.smid + (size_t)e * (D + 1));
}

}  // namespace

void lut_project_device(Kernel k, int K, int D, int n, const double* theta, double* shat, double* smid, double* err2,
                        hipStream_t st) {
  if (K < 1 || K > 6 || D < 1 || D > 6 || K * D < 2) throw Error(SPH_HOA_E_INVALID_ARG, "need 1 <= K, D <= 6, K D >= 2");
  if (n < 2 || n > 65536) throw Error(SPH_HOA_E_INVALID_ARG, "table size must be 2..65536");
  if (!theta || !shat || !smid || !err2) throw Error(SPH_HOA_E_INVALID_ARG, "null table pointer");
  LutProjArgs A{};
  A.kernel = k;
  A.K = K;
  A.D = D;
  A.P = (K + 1) / 2;
  A.n = n;
  A.nb = lut_basis(K, D, A.bk, A.bd);
  gauss_legendre(kLutGL, A.glx, A.glw);
  A.theta = theta;
  A.shat = shat;
  A.smid = smid;
  A.err2 = err2;
  uint32_t* status = nullptr;
  hip_check(hipMallocAsync((void**)&status, sizeof(uint32_t), st), "hipMallocAsync");
  A.status = status;
  uint32_t h_status = 0;
  hipError_t err = hipMemsetAsync(status, 0, sizeof(uint32_t), st);
  if (err == hipSuccess) {
    k_lut_project<<<n, 64, 0, st>>>(A);
    err = hipGetLastError();
  }
  if (err == hipSuccess) err = hipMemcpyAsync(&h_status, status, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  (void)hipFreeAsync(status, st);
  hip_check(err, "k_lut_project");
  if (h_status & 1u) throw Error(SPH_HOA_E_INVALID_ARG, "knot table rows must be positive and increasing");
  if (h_status & 2u) throw Error(SPH_HOA_E_INVALID_ARG, "knot table entry needs too many quadrature nodes");
  if (h_status & 4u) throw Error(SPH_HOA_E_INVALID_ARG, "knot table entry is not a valid set of knots (singular projection)");
}

void project_table_device(Table& T, hipStream_t st) {
  const int n = T.n, P = T.P, D = T.D;
  const size_t nt = (size_t)n * P, ns = (size_t)n * P * (D + 1), nm = (size_t)n * (D + 1);
  double* buf = nullptr;
  hip_check(hipMallocAsync((void**)&buf, (nt + ns + nm + n) * sizeof(double), st), "hipMallocAsync");
  double *d_theta = buf, *d_shat = buf + nt, *d_smid = d_shat + ns, *d_err2 = d_smid + nm;
  T.shat.assign(ns, 0.0);
  T.smid.assign(nm, 0.0);
  T.err2.assign(n, 0.0);
  try {
    hip_check(hipMemcpyAsync(d_theta, T.theta.data(), nt * sizeof(double), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    lut_project_device(T.kernel, T.K, D, n, d_theta, d_shat, d_smid, d_err2, st);
    hip_check(hipMemcpyAsync(T.shat.data(), d_shat, ns * sizeof(double), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hip_check(hipMemcpyAsync(T.smid.data(), d_smid, nm * sizeof(double), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hip_check(hipMemcpyAsync(T.err2.data(), d_err2, n * sizeof(double), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  } catch (...) {
    (void)hipFreeAsync(buf, st);
    throw;
  }
  hip_check(hipFreeAsync(buf, st), "hipFreeAsync");
}

}  // namespace sph
