// Host-side table machinery under AddressSanitizer and UndefinedBehaviorSanitizer: the knot
// optimisation (Sec. 3.4) with its worker threads, the projection and jump conversion (Sec. 3.3,
// Sec. 3.1), the kernel constants and the length quantum (Sec. 4.4), for every kernel and a spread
// of K and D.  Exits non-zero if a result is not finite; the sanitizers abort on any finding.
#include <cmath>
#include <cstdio>
#include <vector>

#include "tables.h"

int main() {
  using sph::Kernel;
  const Kernel kernels[] = {Kernel::Cubic, Kernel::Wendland, Kernel::WendlandC4, Kernel::WendlandC6,
                            Kernel::WendlandGrad, Kernel::WendlandC4Grad, Kernel::WendlandC6Grad};
  const int kd[][2] = {{4, 2}, {3, 3}, {1, 2}, {6, 4}, {5, 2}, {2, 6}};
  int bad = 0;
  for (Kernel k : kernels) {
    const double ka = sph::kernel_kappa(k), kp = sph::kernel_kappa_prime(k);
    if (!(ka > 0 && kp > 0)) ++bad;
    for (const auto& c : kd) {
      const sph::Table t = sph::build_table(k, c[0], c[1], 16, nullptr, 4);
      for (double e : t.err2) bad += !std::isfinite(e);
      for (double x : t.shat) bad += !std::isfinite(x);
      // the same table from its own knots (the given-knots path)
      const sph::Table u = sph::build_table(k, c[0], c[1], 16, t.theta.data(), 3);
      for (size_t i = 0; i < u.shat.size(); ++i) bad += !(u.shat[i] == t.shat[i]);
      for (int D = 1; D <= 6; ++D) bad += !(sph::optimal_tau(k, D, 1e-14, 0.01, 1.0) > 0);
    }
  }
  std::printf("host tables: %d problems\n", bad);
  return bad == 0 ? 0 : 1;
}
