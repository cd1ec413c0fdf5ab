// Host-side tables and quanta: see tables.h.
//
// The projection (Sec. 3.3) solves the normal equations G c = b of the basis
// A~_kd (App. A.1) with inner products by Gauss-Legendre quadrature.  On the
// part of the line inside the kernel support the substitution
// t = Lambda sinh(u) turns sqrt(Lambda^2 + t^2) = Lambda cosh(u) into an entire
// function, so the quadrature converges fast even for rays through the centre.
// The knot optimisation (Sec. 3.4) minimises E^2(theta) with damped Newton
// steps on the gradient dE^2/dtheta_j = -2 <B - S, sum_i c_i dA~_i/dtheta_j>
// (valid because S is the projection for the current knots), in coordinates
// that keep the knots ordered, from several starting shapes; the table keeps
// the best optimum and then retries each entry from its neighbours' optima.
#include "tables.h"

#include "lutmath.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <limits>
#include <stdexcept>
#include <thread>

namespace sph {

namespace {

constexpr double kPi = 3.14159265358979323846;

struct GL {
  std::vector<double> x, w;  // on [-1, 1]
};

GL make_gl(int n) {
  GL g;
  g.x.resize(n);
  g.w.resize(n);
  gauss_legendre(n, g.x.data(), g.w.data());
  return g;
}

const GL& gl16() {
  static const GL g = make_gl(16);
  return g;
}

double kernel_dw(Kernel k, double r) {
  if (r >= kSupport) return 0.0;
  if (k == Kernel::Cubic) {
    if (r < 1.0) return (-12.0 * r + 9.0 * r * r) / (4.0 * kPi);
    return -3.0 * (2.0 - r) * (2.0 - r) / (4.0 * kPi);
  }
  const double a = 1.0 - 0.5 * r, a2 = a * a, a4 = a2 * a2;
  if (k == Kernel::WendlandGrad) return 21.0 / (16.0 * kPi) * (-7.5) * a2;
  if (k == Kernel::WendlandC4Grad) return 495.0 / (256.0 * kPi) * (-35.0) * r * a4;
  if (k == Kernel::WendlandC6Grad) return 1365.0 / (512.0 * kPi) * (-33.0) * r * (1.0 + 3.0 * r) * a4 * a2;
  // derivatives of the factored forms (1 - r/2)^n p(r)
  if (k == Kernel::WendlandC4) return 495.0 / (256.0 * kPi) * (-14.0 / 3.0) * r * (1.0 + 2.5 * r) * a4 * a;
  if (k == Kernel::WendlandC6)
    return 1365.0 / (512.0 * kPi) * (-5.5) * r * (1.0 + r * (3.5 + 4.0 * r)) * a4 * a2 * a;
  return 21.0 / (16.0 * kPi) * (-5.0 * r) * a2 * a;
}

struct Quad {
  std::vector<double> t, w, B;
};

// Quadrature nodes of the inner products (lutmath.h: quad_plan, quad_node).
void build_quad(Kernel k, double lam, const double* theta, int P, Quad& Q) {
  const GL& g = gl16();
  QuadPlan plan;
  quad_plan(k, lam, theta, P, plan);
  const int m = plan.first[plan.nseg];
  Q.t.resize(m);
  Q.w.resize(m);
  Q.B.resize(m);
  for (int i = 0; i < m; ++i) quad_node(k, plan, g.x.data(), g.w.data(), i, &Q.t[i], &Q.w[i], &Q.B[i]);
}

struct Basis {
  int K, D, P;
  std::vector<int> bk, bd;  // index set J (App. A.1)
};

Basis make_basis(int K, int D) {
  Basis b;
  b.K = K;
  b.D = D;
  b.P = (K + 1) / 2;
  int bk[64], bd[64];
  const int n = lut_basis(K, D, bk, bd);
  b.bk.assign(bk, bk + n);
  b.bd.assign(bd, bd + n);
  return b;
}

inline double ipow(double x, int n) { return lut_ipow(x, n); }

// Cholesky solve of the small SPD system; false if not positive definite.
bool chol_solve(std::vector<double>& G, std::vector<double>& x, int n) { return lut_chol_solve(G.data(), x.data(), n); }

struct Proj {
  std::vector<double> c;
  double E2 = 0, B2 = 0;
  std::vector<double> grad;  // dE^2 / dtheta_j
};

// Projection of B_Lambda for knots theta[0..P-1] (positive).
bool project(Kernel k, const Basis& bs, double lam, const double* theta, bool want_grad, Proj& out, Quad& Q) {
  const int P = bs.P, n = (int)bs.bk.size();
  double th[8];
  th[0] = 0.0;
  for (int i = 0; i < P; ++i) th[i + 1] = theta[i];
  for (int i = 0; i < P; ++i)
    if (!(th[i + 1] > th[i])) return false;
  build_quad(k, lam, theta, P, Q);
  const size_t m = Q.t.size();
  std::vector<double> A(n * m);
  for (int i = 0; i < n; ++i)
    for (size_t j = 0; j < m; ++j) A[i * m + j] = basis_val(th, bs.bk[i], bs.bd[i], Q.t[j]);
  std::vector<double> G(n * n, 0.0), b(n, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int l = 0; l <= i; ++l) {
      double s = 0.0;
      for (size_t j = 0; j < m; ++j) s += Q.w[j] * A[i * m + j] * A[l * m + j];
      G[i * n + l] = G[l * n + i] = 2.0 * s;
    }
    double s = 0.0;
    for (size_t j = 0; j < m; ++j) s += Q.w[j] * A[i * m + j] * Q.B[j];
    b[i] = 2.0 * s;
  }
  if (!chol_solve(G, b, n)) return false;
  out.c = b;
  double e2 = 0.0, b2 = 0.0;
  std::vector<double> R(m);
  for (size_t j = 0; j < m; ++j) {
    double S = 0.0;
    for (int i = 0; i < n; ++i) S += out.c[i] * A[i * m + j];
    R[j] = Q.B[j] - S;
    e2 += Q.w[j] * R[j] * R[j];
    b2 += Q.w[j] * Q.B[j] * Q.B[j];
  }
  out.E2 = 2.0 * e2;
  out.B2 = 2.0 * b2;
  if (want_grad) {
    out.grad.assign(P, 0.0);
    for (int jv = 1; jv <= P; ++jv) {
      double g = 0.0;
      for (size_t j = 0; j < m; ++j) {
        const double t = Q.t[j];
        double dS = 0.0;
        for (int i = 0; i < n; ++i) {
          const int kk = bs.bk[i], d = bs.bd[i];
          const double a = th[kk - 1], bb = th[kk];
          if (!(t > a && t < bb)) continue;
          const double z = (t - a) / (bb - a);
          if (jv == kk) dS += out.c[i] * d / (bb - a) * ipow(z, d);
          else if (jv == kk - 1) dS += out.c[i] * d / (bb - a) * ipow(z, d - 1) * (1.0 - z);
        }
        g += Q.w[j] * R[j] * dS;
      }
      out.grad[jv - 1] = -4.0 * g;
    }
  }
  return true;
}

// Objective in p-coordinates: y_1 = exp(p_1), y_i = y_{i-1} + exp(p_i), theta = s y.
struct Objective {
  Kernel k;
  const Basis& bs;
  double lam, s, scale;
  Quad Q;
  Proj pr;
  bool eval(const double* p, double* f, double* g) {
    const int P = bs.P;
    double y[4], th[4];
    double acc = 0.0;
    for (int i = 0; i < P; ++i) {
      acc += std::exp(p[i]);
      y[i] = acc;
      th[i] = s * y[i];
    }
    if (!project(k, bs, lam, th, g != nullptr, pr, Q)) {
      *f = std::numeric_limits<double>::infinity();
      if (g)
        for (int i = 0; i < P; ++i) g[i] = 0.0;
      return false;
    }
    *f = pr.E2 / scale;
    if (g) {
      double run = 0.0;
      for (int i = P - 1; i >= 0; --i) {
        run += pr.grad[i] * s;
        g[i] = run * std::exp(p[i]) / scale;
      }
    }
    return true;
  }
};

bool solve_small(double* H, double* g, double* x, int n) {
  std::vector<double> Gm(H, H + n * n), v(g, g + n);
  if (!chol_solve(Gm, v, n)) return false;
  for (int i = 0; i < n; ++i) x[i] = v[i];
  return true;
}

// Local minimisation from y0 (normalised knots).
void local_opt(Kernel k, const Basis& bs, double lam, const double* y0, double* y_out, double* e2_out) {
  const int P = bs.P;
  const double s = std::sqrt((kSupport - lam) * (kSupport + lam));
  Objective ob{k, bs, lam, s, 1.0, {}, {}};
  double th0[4];
  for (int i = 0; i < P; ++i) th0[i] = s * y0[i];
  {
    Proj tmp;
    Quad q2;
    project(k, bs, lam, th0, false, tmp, q2);
    ob.scale = tmp.B2 > 0 ? tmp.B2 : 1.0;
  }
  double p[4], g[4], f;
  double prev = 0.0;
  for (int i = 0; i < P; ++i) {
    p[i] = std::log(y0[i] - prev);
    prev = y0[i];
  }
  ob.eval(p, &f, g);
  auto hessian = [&](const double* pp, double* H) {
    const double h = 1e-5;
    for (int i = 0; i < P; ++i) {
      double pa[4], pb[4], ga[4], gb[4], fa, fb;
      for (int j = 0; j < P; ++j) pa[j] = pb[j] = pp[j];
      pa[i] += h;
      pb[i] -= h;
      ob.eval(pa, &fa, ga);
      ob.eval(pb, &fb, gb);
      for (int j = 0; j < P; ++j) H[j * P + i] = (ga[j] - gb[j]) / (2 * h);
    }
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < i; ++j) H[i * P + j] = H[j * P + i] = 0.5 * (H[i * P + j] + H[j * P + i]);
  };
  bool converged = false;
  for (int it = 0; it < 60 && !converged; ++it) {
    double H[16], step[4];
    hessian(p, H);
    if (!solve_small(H, g, step, P)) break;
    double mx = 0.0;
    for (int i = 0; i < P; ++i) mx = std::max(mx, std::fabs(step[i]));
    double a = std::min(1.0, 1.0 / std::max(1e-300, mx));
    bool ok = false;
    double pn[4], gn[4], fn = 0;
    while (a > 1e-4) {
      for (int i = 0; i < P; ++i) pn[i] = p[i] - a * step[i];
      ob.eval(pn, &fn, gn);
      if (fn <= f + 1e-15 * std::fabs(f)) {
        ok = true;
        break;
      }
      a *= 0.5;
    }
    if (!ok) break;
    for (int i = 0; i < P; ++i) {
      p[i] = pn[i];
      g[i] = gn[i];
    }
    f = fn;
    if (a * mx < 1e-12) converged = true;
  }
  if (!converged) {
    // BFGS with a backtracking line search, then a few Newton steps
    double Hinv[16] = {0};
    for (int i = 0; i < P; ++i) Hinv[i * P + i] = 1.0;
    for (int it = 0; it < 500; ++it) {
      double d[4];
      for (int i = 0; i < P; ++i) {
        d[i] = 0.0;
        for (int j = 0; j < P; ++j) d[i] -= Hinv[i * P + j] * g[j];
      }
      double slope = 0.0;
      for (int i = 0; i < P; ++i) slope += d[i] * g[i];
      if (!(slope < 0.0)) {
        for (int i = 0; i < P * P; ++i) Hinv[i] = (i % (P + 1) == 0) ? 1.0 : 0.0;
        for (int i = 0; i < P; ++i) d[i] = -g[i];
        slope = 0.0;
        for (int i = 0; i < P; ++i) slope += d[i] * g[i];
      }
      double a = 1.0, pn[4], gn[4], fn = 0;
      bool ok = false;
      for (int ls = 0; ls < 60; ++ls) {
        for (int i = 0; i < P; ++i) pn[i] = p[i] + a * d[i];
        ob.eval(pn, &fn, gn);
        if (fn <= f + 1e-4 * a * slope) {
          ok = true;
          break;
        }
        a *= 0.5;
      }
      if (!ok) break;
      double sv[4], yv[4], sy = 0.0;
      for (int i = 0; i < P; ++i) {
        sv[i] = pn[i] - p[i];
        yv[i] = gn[i] - g[i];
        sy += sv[i] * yv[i];
      }
      for (int i = 0; i < P; ++i) {
        p[i] = pn[i];
        g[i] = gn[i];
      }
      const double df = f - fn;
      f = fn;
      if (sy > 1e-300) {
        double Hy[4];
        for (int i = 0; i < P; ++i) {
          Hy[i] = 0.0;
          for (int j = 0; j < P; ++j) Hy[i] += Hinv[i * P + j] * yv[j];
        }
        double yHy = 0.0;
        for (int i = 0; i < P; ++i) yHy += yv[i] * Hy[i];
        for (int i = 0; i < P; ++i)
          for (int j = 0; j < P; ++j)
            Hinv[i * P + j] += (sy + yHy) * sv[i] * sv[j] / (sy * sy) - (Hy[i] * sv[j] + sv[i] * Hy[j]) / sy;
      }
      double gn2 = 0.0;
      for (int i = 0; i < P; ++i) gn2 = std::max(gn2, std::fabs(g[i]));
      if (gn2 < 1e-14 || df <= 1e-18 * std::fabs(f)) break;
    }
    for (int it = 0; it < 8; ++it) {
      double H[16], step[4], pn[4], gn[4], fn;
      hessian(p, H);
      if (!solve_small(H, g, step, P)) break;
      for (int i = 0; i < P; ++i) pn[i] = p[i] - step[i];
      ob.eval(pn, &fn, gn);
      if (!(fn <= f * (1 + 1e-14))) break;
      double mx = 0.0;
      for (int i = 0; i < P; ++i) {
        mx = std::max(mx, std::fabs(step[i]));
        p[i] = pn[i];
        g[i] = gn[i];
      }
      f = fn;
      if (mx < 1e-12) break;
    }
  }
  double acc = 0.0;
  for (int i = 0; i < P; ++i) {
    acc += std::exp(p[i]);
    y_out[i] = acc;
  }
  double th[4], fe;
  for (int i = 0; i < P; ++i) th[i] = s * y_out[i];
  Proj pr;
  Quad q3;
  if (project(k, bs, lam, th, false, pr, q3)) fe = pr.E2;
  else fe = std::numeric_limits<double>::infinity();
  *e2_out = fe;
}

void jumps_from_coeffs(const Basis& bs, const double* theta, const std::vector<double>& c, double* shat,
                       double* smid) {
  lut_jumps(bs.K, bs.D, bs.bk.data(), bs.bd.data(), (int)c.size(), theta, c.data(), shat, smid);
}

}  // namespace

double kernel_w(Kernel k, double r) {
  if (r < 0) r = -r;
  if (r >= kSupport) return 0.0;
  return kernel_w_edge(k, r, kSupport - r);
}

double kernel_w0(Kernel k) { return kernel_w(k, 0.0); }

double kernel_kappa(Kernel k) {
  // 4 pi int_0^q (t w(t))^2 dt; the integrand is a polynomial on [0,1] and [1,2]
  const GL& g = gl16();
  double s = 0.0;
  for (int piece = 0; piece < 2; ++piece) {
    const double a = piece, b = piece + 1.0;
    for (size_t i = 0; i < g.x.size(); ++i) {
      const double t = 0.5 * (b - a) * g.x[i] + 0.5 * (b + a);
      const double v = t * kernel_w(k, t);
      s += 0.5 * (b - a) * g.w[i] * v * v;
    }
  }
  return std::sqrt(4.0 * kPi * s);
}

double kernel_kappa_prime(Kernel k) {
  // int_0^q Lambda int_R (dB/dt)^2 dt dLambda = (1/2pi) int_{R^3} (d f/dz)^2 dV
  //   = (1/2pi)(1/3) int |grad f|^2 dV = (2/3) int_0^q r^2 w'(r)^2 dr  (f = w(|x|), isotropic)
  const GL& g = gl16();
  double s = 0.0;
  for (int piece = 0; piece < 2; ++piece) {
    const double a = piece, b = piece + 1.0;
    for (size_t i = 0; i < g.x.size(); ++i) {
      const double r = 0.5 * (b - a) * g.x[i] + 0.5 * (b + a);
      const double v = r * kernel_dw(k, r);
      s += 0.5 * (b - a) * g.w[i] * v * v;
    }
  }
  return std::sqrt(2.0 / 3.0 * s);
}

// Starting shapes y = theta / s: a grid over the plausible region, because neighbouring
// local optima of E^2 can differ by about one percent.
std::vector<double> default_starts(int P) {
  std::vector<double> s;
  if (P == 1) {
    for (int i = 0; i < 9; ++i) s.push_back(0.3 + 0.1 * i);
  } else if (P == 2) {
    const double a[5] = {0.2, 0.3, 0.4, 0.5, 0.6}, b[5] = {0.7, 0.8, 0.9, 1.0, 1.1};
    for (double y1 : a)
      for (double y2 : b) {
        s.push_back(y1);
        s.push_back(y2);
      }
  } else if (P == 3) {
    const double a[3] = {0.15, 0.3, 0.45}, b[3] = {0.5, 0.65, 0.8}, c[3] = {0.9, 1.0, 1.1};
    for (double y1 : a)
      for (double y2 : b)
        for (double y3 : c) {
          s.push_back(y1);
          s.push_back(y2);
          s.push_back(y3);
        }
  } else {
    throw std::invalid_argument("K <= 6");
  }
  return s;
}

void optimal_knots(Kernel k, int K, int D, double lambda, const std::vector<double>& starts, double* theta_out,
                   double* err2_out) {
  const Basis bs = make_basis(K, D);
  const int P = bs.P;
  const double s = std::sqrt((kSupport - lambda) * (kSupport + lambda));
  double best = std::numeric_limits<double>::infinity();
  double by[4] = {0, 0, 0, 0};
  for (size_t st = 0; st + P <= starts.size(); st += P) {
    double y[4], e2;
    local_opt(k, bs, lambda, &starts[st], y, &e2);
    if (e2 < best) {
      best = e2;
      for (int i = 0; i < P; ++i) by[i] = y[i];
    }
  }
  for (int i = 0; i < P; ++i) theta_out[i] = s * by[i];
  *err2_out = best;
}

double project_jumps(Kernel k, int K, int D, double lambda, const double* theta, double* shat_rows,
                     double* smid_row) {
  const Basis bs = make_basis(K, D);
  Proj pr;
  Quad Q;
  if (!project(k, bs, lambda, theta, false, pr, Q)) return std::numeric_limits<double>::infinity();
  jumps_from_coeffs(bs, theta, pr.c, shat_rows, smid_row);
  return pr.E2;
}

Table build_table(Kernel k, int K, int D, int n, const double* given_theta, int n_threads, bool project) {
  Table T;
  T.K = K;
  T.D = D;
  T.P = (K + 1) / 2;
  T.n = n;
  T.kernel = k;
  const int P = T.P;
  T.theta.assign((size_t)n * P, 0.0);
  T.shat.assign((size_t)n * P * (D + 1), 0.0);
  T.smid.assign((size_t)n * (D + 1), 0.0);
  T.err2.assign(n, 0.0);
  auto lam_of = [&](int i) { return (i + 0.5) * kSupport / n; };
  auto s_of = [&](int i) {
    const double l = lam_of(i);
    return std::sqrt((kSupport - l) * (kSupport + l));
  };
  auto parallel = [&](auto fn) {
    std::atomic<int> next(0);
    std::vector<std::thread> th;
    const int nt = std::max(1, n_threads);
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&]() {
        for (int i = next++; i < n; i = next++) fn(i);
      });
    for (auto& x : th) x.join();
  };
  if (given_theta) {
    std::copy(given_theta, given_theta + (size_t)n * P, T.theta.begin());
  } else {
    // pass 1: fixed starting shapes; pass 2: neighbours' optima as extra starts
    const std::vector<double> starts = default_starts(P);
    std::vector<double> y1((size_t)n * P), e1(n);
    parallel([&](int i) {
      double th[4], e2;
      optimal_knots(k, K, D, lam_of(i), starts, th, &e2);
      for (int j = 0; j < P; ++j) y1[(size_t)i * P + j] = th[j] / s_of(i);
      e1[i] = e2;
    });
    parallel([&](int i) {
      std::vector<double> st;
      for (int j = 0; j < P; ++j) st.push_back(y1[(size_t)i * P + j]);
      if (i > 0)
        for (int j = 0; j < P; ++j) st.push_back(y1[(size_t)(i - 1) * P + j]);
      if (i + 1 < n)
        for (int j = 0; j < P; ++j) st.push_back(y1[(size_t)(i + 1) * P + j]);
      double th[4], e2;
      optimal_knots(k, K, D, lam_of(i), st, th, &e2);
      if (e2 <= e1[i]) {
        for (int j = 0; j < P; ++j) T.theta[(size_t)i * P + j] = th[j];
      } else {
        for (int j = 0; j < P; ++j) T.theta[(size_t)i * P + j] = s_of(i) * y1[(size_t)i * P + j];
      }
    });
  }
  if (!project) return T;
  parallel([&](int i) {
    T.err2[i] = project_jumps(k, K, D, lam_of(i), &T.theta[(size_t)i * P], &T.shat[(size_t)i * P * (D + 1)],
                              &T.smid[(size_t)i * (D + 1)]);
  });
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(T.err2[i])) throw std::runtime_error("knot table entry is not a valid set of knots");
  return T;
}

double optimal_tau(Kernel k, int D, double sigma, double h_repr, double phi_repr) {
  // minimiser of Q_D(x, r) over x, r = sigma / phi_repr (App. A.5): root of
  // dQ^2/dx = kp^2 x / (8 ka^2) - sum_{d=1..D} d q^{2d+3} / (4 ka^2 (2d+1)(2d+3)) r^2 / x^{2d+1},
  // strictly increasing in x; multiply by 8 ka^2 x / kp^2 > 0 (same sign):
  // h(x) = x^2 - (2 / kp^2) sum_d d q^{2d+3} / ((2d+1)(2d+3)) r^2 x^{-2d}
  const double ka = kernel_kappa(k), kp = kernel_kappa_prime(k);
  (void)ka;
  const double r = sigma / phi_repr;
  auto h = [&](double lx) {
    const double x = std::exp(lx);
    double s = 0.0;
    for (int d = 1; d <= D; ++d)
      s += d * std::pow(kSupport, 2 * d + 3) / ((2.0 * d + 1) * (2.0 * d + 3)) * r * r * std::exp(-2.0 * d * lx);
    return x * x - 2.0 / (kp * kp) * s;
  };
  double lo = -700.0, hi = 10.0;
  while (h(hi) <= 0.0) hi += 10.0;
  for (int it = 0; it < 400; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (h(mid) > 0.0) hi = mid;
    else lo = mid;
  }
  return h_repr * std::exp(hi);
}

}  // namespace sph
