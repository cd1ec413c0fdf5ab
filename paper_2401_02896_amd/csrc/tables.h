// Host-side preparation of the per-configuration tables and quanta.
//
// Sec. 3.1: a look-up table over equidistant distance parameters Lambda holds,
// for each entry, the optimal positive knots theta_k (Sec. 3.4) and the
// localized difference coefficients of the L2-optimal approximation of
// B_Lambda(t) = w(sqrt(Lambda^2 + t^2)) (Sec. 3.3).  Sec. 4.4 chooses the
// quanta.  This is setup work done once per (kernel, K, D, table size).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sph {

// The *Grad kernels are g(r) = -w'(r) / r of the Wendland kernel named: the radial factor of a
// particle's gradient, h^-4 w'(r) y / r with y = (x - chi) / h.  Along a ray the gradient's part
// across the ray is a field of g (Sec. 6: features generated additively by the particles).
enum class Kernel : int {
  Cubic = 0,
  Wendland = 1,
  WendlandC4 = 2,
  WendlandC6 = 3,
  WendlandGrad = 4,
  WendlandC4Grad = 5,
  WendlandC6Grad = 6
};

constexpr double kSupport = 2.0;  // q for both kernels

struct Table {
  int K = 0, D = 0, P = 0, n = 0;
  Kernel kernel = Kernel::Cubic;
  std::vector<double> theta;  // [n][P]
  std::vector<double> shat;   // [n][P][D+1], jump at +theta_k localized there
  std::vector<double> smid;   // [n][D+1], jump at 0 for even K
  std::vector<double> err2;   // [n] squared L2 error of the approximation
};

// Kernel value w(r).
double kernel_w(Kernel k, double r);
double kernel_w0(Kernel k);
// kappa = (4 pi int t^2 w^2)^(1/2) and kappa' (Sec. 4.4).
double kernel_kappa(Kernel k);
double kernel_kappa_prime(Kernel k);

// Optimal knots for one Lambda from the given start points (normalised y = theta / s) and
// returns theta and E^2.  `starts` holds P values per start.
void optimal_knots(Kernel k, int K, int D, double lambda, const std::vector<double>& starts,
                   double* theta_out, double* err2_out);
std::vector<double> default_starts(int P);

// Projection coefficients for fixed knots; fills the jump coefficients. Returns E^2 (inf if singular).
double project_jumps(Kernel k, int K, int D, double lambda, const double* theta, double* shat_rows,
                     double* smid_row);

// Full table (optimisation unless `given_theta` is non-null); with project = false the jump
// coefficients and errors are left for the device projection (project_table_device).
Table build_table(Kernel k, int K, int D, int n, const double* given_theta, int n_threads, bool project = true);

// Length quantum minimising Q_D(tau / h_repr, sigma / phi_repr).
double optimal_tau(Kernel k, int D, double sigma, double h_repr, double phi_repr);

}  // namespace sph
