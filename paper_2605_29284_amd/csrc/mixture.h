// Spatially weighted mixtures of stationary components (GPU helpers).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace krig {

constexpr int MIX_MAX = 8;  // components per call

// beta[b][i] = lam[i] * alpha[b][i], b < B, i < n
hipError_t mix_scale_coef(const double* alpha, const double* lam, int n, int B, double* beta, hipStream_t st);

// out[b][q] = sum_{c < C} lam[c][q] * comp[c][b][q] in that order, FP64 accumulation,
// rounded once to the output type; q < npix = m1 m2.
struct MixArgs {
  const void* comp[MIX_MAX];  // [B][npix] each, float or double
  const double* lam;          // [C][npix]
  int C;
  int64_t npix;
  int B;
  void* out;                  // [B][npix]
};
hipError_t mix_combine(const MixArgs& a, bool f32, hipStream_t st);

}  // namespace krig
