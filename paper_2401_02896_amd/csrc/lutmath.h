// Arithmetic of the table projection (Sec. 3.3) shared by the host table builder and the device
// projection kernel: kernel values, the candidate basis (App. A.1), the quadrature plan of the
// inner products, the Cholesky solve of the normal equations and the conversion of the projection
// coefficients into localized jump coefficients (Sec. 3.1).  Every function is written for raw
// arrays and runs on the host and on the device with the same operations in the same order.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "tables.h"

namespace sph {

constexpr double kLutPi = 3.14159265358979323846;

// n-point Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on the three-term Legendre
// recurrence from the usual cosine estimates (host).
inline void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kLutPi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        p0 = 1.0;
        p1 = z;
        for (int k = 2; k <= n; ++k) {
          const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        break;
      }
    }
  }
}

// w with q - r supplied separately for the outermost polynomial piece.
__host__ __device__ inline double kernel_w_edge(Kernel k, double r, double e) {
  if (e <= 0.0) return 0.0;
  if (k == Kernel::Cubic) {
    if (r < 1.0) return (4.0 - 6.0 * r * r + 3.0 * r * r * r) / (4.0 * kLutPi);
    return e * e * e / (4.0 * kLutPi);
  }
  const double h = 0.5 * e;  // 1 - r / 2
  const double h2 = h * h, h4 = h2 * h2;
  // g = -w'/r of the Wendland kernels, (1 - r/2)^(n-1) times a polynomial
  if (k == Kernel::WendlandGrad) return 21.0 / (16.0 * kLutPi) * 5.0 * h2 * h;
  if (k == Kernel::WendlandC4Grad) return 495.0 / (256.0 * kLutPi) * (14.0 / 3.0) * h4 * h * (1.0 + 2.5 * r);
  if (k == Kernel::WendlandC6Grad)
    return 1365.0 / (512.0 * kLutPi) * 5.5 * h4 * h2 * h * (1.0 + r * (3.5 + 4.0 * r));
  if (k == Kernel::WendlandC4) return 495.0 / (256.0 * kLutPi) * h4 * h2 * (1.0 + r * (3.0 + r * (35.0 / 12.0)));
  if (k == Kernel::WendlandC6)
    return 1365.0 / (512.0 * kLutPi) * h4 * h4 * (1.0 + r * (4.0 + r * (25.0 / 4.0 + r * 4.0)));
  return 21.0 / (16.0 * kLutPi) * h4 * (1.0 + 2.0 * r);
}

__host__ __device__ inline double lut_ipow(double x, int n) {
  double r = 1.0;
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}

// The index set J of the basis (App. A.1): (k, d) for k = 1..P, d = 1..D, without (1, odd d) for
// odd K.  Fills bk/bd (room for P * D entries) and returns |J| = floor(K D / 2).
__host__ __device__ inline int lut_basis(int K, int D, int* bk, int* bd) {
  const int P = (K + 1) / 2;
  int n = 0;
  for (int k = 1; k <= P; ++k)
    for (int d = 1; d <= D; ++d)
      if (!(K % 2 == 1 && k == 1 && d % 2 == 1)) {
        bk[n] = k;
        bd[n] = d;
        ++n;
      }
  return n;
}

// A~_kd(t) for t >= 0 with th[0] = 0.
__host__ __device__ inline double basis_val(const double* th, int k, int d, double t) {
  const double a = th[k - 1], b = th[k];
  if (t <= a) return 1.0;
  if (t >= b) return 0.0;
  return 1.0 - lut_ipow((t - a) / (b - a), d);
}

// Gauss-Legendre nodes of the inner products on [0, max(theta_P, s)], s = sqrt(q^2 - Lambda^2):
// the interval is split at 0, s, the knots and the cubic spline's breakpoint; a piece inside the
// support is integrated in u with t = Lambda sinh(u) (sqrt(Lambda^2 + t^2) = Lambda cosh(u) is
// entire in u) over sub-intervals of at most 0.5, a piece beyond s directly; 16 points per
// sub-interval.  Node j of sub-interval i of piece c has index first[c] + 16 i + j.
constexpr int kLutGL = 16;
struct QuadPlan {
  int nseg;
  double a[8], b[8];
  double ua[8], ub[8];  // sinh pieces: u range
  int sinh_piece[8];
  int m[8];             // sub-intervals
  int first[9];         // first node of each piece
  double s, lam;
};

__host__ __device__ inline void quad_plan(Kernel k, double lam, const double* theta, int P, QuadPlan& Q) {
  const double s = sqrt((kSupport - lam) * (kSupport + lam));
  double cuts[8];
  int nc = 0;
  cuts[nc++] = 0.0;
  cuts[nc++] = s;
  for (int i = 0; i < P; ++i) cuts[nc++] = theta[i];
  if (k == Kernel::Cubic && lam < 1.0) cuts[nc++] = sqrt((1.0 - lam) * (1.0 + lam));
  for (int i = 1; i < nc; ++i)  // insertion sort (at most 6 values)
    for (int j = i; j > 0 && cuts[j - 1] > cuts[j]; --j) {
      const double t = cuts[j];
      cuts[j] = cuts[j - 1];
      cuts[j - 1] = t;
    }
  Q.s = s;
  Q.lam = lam;
  Q.nseg = 0;
  Q.first[0] = 0;
  for (int c = 0; c + 1 < nc; ++c) {
    const double a = cuts[c], b = cuts[c + 1];
    if (!(b > a)) continue;
    const int g = Q.nseg;
    Q.a[g] = a;
    Q.b[g] = b;
    if (b <= s && lam > 0.0) {
      Q.sinh_piece[g] = 1;
      Q.ua[g] = asinh(a / lam);
      Q.ub[g] = asinh(b / lam);
      const double mm = ceil((Q.ub[g] - Q.ua[g]) / 0.5);
      Q.m[g] = mm < 1.0 ? 1 : (int)mm;
    } else {
      Q.sinh_piece[g] = 0;
      Q.ua[g] = Q.ub[g] = 0.0;
      Q.m[g] = 1;
    }
    Q.first[g + 1] = Q.first[g] + kLutGL * Q.m[g];
    ++Q.nseg;
  }
}

// Node idx of the plan: position t, weight w and B_Lambda(t) = w(sqrt(Lambda^2 + t^2)).
__host__ __device__ inline void quad_node(Kernel k, const QuadPlan& Q, const double* glx, const double* glw, int idx,
                                          double* t_out, double* w_out, double* B_out) {
  int g = 0;
  while (idx >= Q.first[g + 1]) ++g;
  const int rel = idx - Q.first[g];
  const int j = rel / kLutGL, i = rel % kLutGL;
  double t, w;
  if (Q.sinh_piece[g]) {
    const double ua = Q.ua[g], ub = Q.ub[g];
    const int m = Q.m[g];
    const double u0 = ua + (ub - ua) * j / m, u1 = ua + (ub - ua) * (j + 1) / m;
    const double hw = 0.5 * (u1 - u0), mid = 0.5 * (u1 + u0);
    const double u = hw * glx[i] + mid;
    t = Q.lam * sinh(u);
    w = hw * glw[i] * Q.lam * cosh(u);
  } else {
    const double a = Q.a[g], b = Q.b[g];
    const double hw = 0.5 * (b - a), mid = 0.5 * (b + a);
    t = hw * glx[i] + mid;
    w = hw * glw[i];
  }
  double B = 0.0;
  if (t < Q.s) {
    const double r = sqrt(Q.lam * Q.lam + t * t);
    const double e = (Q.s - t) * (Q.s + t) / (kSupport + r);
    B = kernel_w_edge(k, r, e);
  }
  *t_out = t;
  *w_out = w;
  *B_out = B;
}

// Cholesky solve of the small SPD system G x = x (n x n, row-major, overwritten); false if G is
// not positive definite.
__host__ __device__ inline bool lut_chol_solve(double* G, double* x, int n) {
  for (int j = 0; j < n; ++j) {
    double s = G[j * n + j];
    for (int k = 0; k < j; ++k) s -= G[j * n + k] * G[j * n + k];
    if (!(s > 0.0)) return false;
    const double l = sqrt(s);
    G[j * n + j] = l;
    for (int i = j + 1; i < n; ++i) {
      double v = G[i * n + j];
      for (int k = 0; k < j; ++k) v -= G[i * n + k] * G[j * n + k];
      G[i * n + j] = v / l;
    }
  }
  for (int i = 0; i < n; ++i) {
    double v = x[i];
    for (int k = 0; k < i; ++k) v -= G[i * n + k] * x[k];
    x[i] = v / G[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double v = x[i];
    for (int k = i + 1; k < n; ++k) v -= G[k * n + i] * x[k];
    x[i] = v / G[i * n + i];
  }
  return true;
}

// Jump coefficients of the projection with coefficients c over the index set (bk, bd, n entries):
//   at +theta_k (k = 1..P): s_kd = sum_{i in J: k_i = k, d_i >= d} c_i C(d_i, d) / Delta_k^d
//                                  - sum_{i in J: k_i = k + 1, d_i = d} c_i / Delta_{k+1}^d
//   at 0 (even K, odd d):   s_0d = -2 sum_{i in J: k_i = 1, d_i = d} c_i / theta_1^d
// (the piece on [theta_{k-1}, theta_k] is sum_{k_i > k} c_i + sum_{k_i = k} c_i (1 - z^{d_i})).
// shat: [P][D + 1]; smid: [D + 1].
__host__ __device__ inline void lut_jumps(int K, int D, const int* bk, const int* bd, int n, const double* theta,
                                          const double* c, double* shat, double* smid) {
  const int P = (K + 1) / 2;
  double th[8];
  th[0] = 0.0;
  for (int i = 0; i < P; ++i) th[i + 1] = theta[i];
  auto binom = [](int nn, int r) {
    double v = 1.0;
    for (int i = 1; i <= r; ++i) v = v * (nn - r + i) / i;
    return v;
  };
  for (int k = 1; k <= P; ++k) {
    const double dk = th[k] - th[k - 1];
    const double dk1 = (k < P) ? th[k + 1] - th[k] : 1.0;
    for (int d = 0; d <= D; ++d) {
      double v = 0.0;
      if (d >= 1) {
        for (int i = 0; i < n; ++i) {
          if (bk[i] == k && bd[i] >= d) v += c[i] * binom(bd[i], d) / lut_ipow(dk, d);
          if (k < P && bk[i] == k + 1 && bd[i] == d) v -= c[i] / lut_ipow(dk1, d);
        }
      }
      shat[(k - 1) * (D + 1) + d] = v;
    }
  }
  for (int d = 0; d <= D; ++d) {
    double v = 0.0;
    if (K % 2 == 0 && d % 2 == 1)
      for (int i = 0; i < n; ++i)
        if (bk[i] == 1 && bd[i] == d) v += -2.0 * c[i] / lut_ipow(th[1], d);
    smid[d] = v;
  }
}

}  // namespace sph
