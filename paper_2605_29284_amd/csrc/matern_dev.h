// Matern covariance on the device: k(d) = sigma2 * phi(d / rho) with the paper's
// phi(d) = d^nu K_nu(d) / (2^(nu-1) Gamma(nu)) (eq. Matern1, range as divisor),
// in the elementary closed forms available for nu = 1/2, 3/2, 5/2, and for nu = 1
// (phi(r) = r K_1(r), no elementary form) by quadrature.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace krig {

struct MaternDev {
  double sigma2, rho, tau2;
  int kind;  // 0: nu = 1/2, 1: nu = 3/2, 2: nu = 5/2, 3: nu = 1
};

// r K_1(r) from K_1(r) = int_0^inf exp(-r cosh t) cosh t dt (DLMF 10.32.9) by the
// trapezoidal rule in t.  The integrand is analytic in a strip around the real axis and
// decays doubly exponentially, so the rule converges geometrically: step 0.05 (shrunk as
// 1/sqrt(r) beyond r = 30, where the strip bound grows like exp(r (1 - cos a))), terms
// until r (cosh t - 1) > 40, with cosh t - 1 formed as 2 sinh^2(t/2) (no cancellation).
// About 1e-15 relative error against a reference K_1 for r in [1e-8, 60]; 30 to ~460
// terms, up to ~14000 as r approaches the smallest doubles.
__host__ __device__ inline double matern_phi_nu1(double r) {
  if (!(r > 0.0)) return 1.0;
  if (r > 700.0) return 0.0;  // r K_1(r) < 1e-302
  const double h = r <= 30.0 ? 0.05 : 0.05 * sqrt(30.0 / r);
  double s = 0.5;  // the t = 0 term, halved
  for (int k = 1; k < 100000; ++k) {
    const double sh = sinh(0.5 * k * h);
    const double e = 2.0 * r * sh * sh;
    if (e > 40.0) break;
    s += exp(-e) * (1.0 + 2.0 * sh * sh);
  }
  return r * exp(-r) * h * s;
}

__host__ __device__ inline double matern_phi(double r, int kind) {
  if (kind == 3) return matern_phi_nu1(r);
  const double e = exp(-r);
  if (kind == 0) return e;
  if (kind == 1) return (1.0 + r) * e;
  return (1.0 + r + r * r * (1.0 / 3.0)) * e;
}

__host__ __device__ inline double matern_cov(double d, const MaternDev& m) {
  return m.sigma2 * matern_phi(d / m.rho, m.kind);
}

}  // namespace krig
