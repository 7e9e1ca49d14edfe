// Matern covariance on the device: k(d) = sigma2 * phi(d / rho) with the paper's
// phi(d) = d^nu K_nu(d) / (2^(nu-1) Gamma(nu)) (eq. Matern1, range as divisor),
// in the elementary closed forms available for nu = 1/2, 3/2, 5/2.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace krig {

struct MaternDev {
  double sigma2, rho, tau2;
  int kind;  // 0: nu = 1/2, 1: nu = 3/2, 2: nu = 5/2
};

__host__ __device__ inline double matern_phi(double r, int kind) {
  const double e = exp(-r);
  if (kind == 0) return e;
  if (kind == 1) return (1.0 + r) * e;
  return (1.0 + r + r * r * (1.0 / 3.0)) * e;
}

__host__ __device__ inline double matern_cov(double d, const MaternDev& m) {
  return m.sigma2 * matern_phi(d / m.rho, m.kind);
}

}  // namespace krig
