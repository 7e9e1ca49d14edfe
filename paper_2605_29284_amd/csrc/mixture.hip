// Nonstationary covariance as a spatially weighted sum of stationary components (the
// closing discussion of the paper): each component is a stationary rapid prediction of
// the coefficients lam_c(s_i) alpha_i, and the results are combined on the grid with
// the weight functions lam_c.
#include "mixture.h"

namespace krig {

__global__ void __launch_bounds__(256) k_mix_scale(const double* __restrict__ alpha, const double* __restrict__ lam,
                                                   int n, int64_t tot, double* __restrict__ beta) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < tot) beta[idx] = lam[idx % n] * alpha[idx];
}

hipError_t mix_scale_coef(const double* alpha, const double* lam, int n, int B, double* beta, hipStream_t st) {
  const int64_t tot = (int64_t)n * B;
  if (tot <= 0) return hipSuccess;
  k_mix_scale<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(alpha, lam, n, tot, beta);
  return hipGetLastError();
}

template <typename TS>
__global__ void __launch_bounds__(256) k_mix_combine(MixArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.npix * a.B) return;
  const int64_t q = idx % a.npix;
  double acc = 0.0;
  for (int c = 0; c < a.C; ++c) acc += a.lam[c * a.npix + q] * (double)reinterpret_cast<const TS*>(a.comp[c])[idx];
  reinterpret_cast<TS*>(a.out)[idx] = (TS)acc;
}

hipError_t mix_combine(const MixArgs& a, bool f32, hipStream_t st) {
  const int64_t tot = a.npix * a.B;
  if (tot <= 0) return hipSuccess;
  if (a.C < 1 || a.C > MIX_MAX) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((tot + 255) / 256);
  if (f32)
    k_mix_combine<float><<<grid, 256, 0, st>>>(a);
  else
    k_mix_combine<double><<<grid, 256, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace krig
