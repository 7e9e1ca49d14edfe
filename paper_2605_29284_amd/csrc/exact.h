// Exact kriging predictions (eq. predictionh): the dense cross-covariance product
// sum_i k(s - s_i) c_i that the rapid method approximates, evaluated directly.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "matern_dev.h"
#include "setup.h"

namespace krig {

struct ExactArgs {
  const double* sites;  // [n][2] FP64
  int n;
  const double* alpha;  // coefficients [B][n] FP64, field pitch alpha_fs
  int64_t alpha_fs;
  const double* pts;    // [npts][2] FP64 evaluation points, or nullptr for the grid nodes of g
  int npts;
  GridDev g;            // node (a, b) = (x0 + a dx, y0 + b dy), a < m1, b < m2, b fastest
  MaternDev mt;         // k without the nugget
  void* out;            // [B][points] (float or double), field pitch out_fs
  int64_t out_fs;
};

// out[b][j] = sum_{i < n} k(|p_j - s_i|) alpha[b][i] in FP64, summed in site order and
// rounded once.  hipErrorInvalidValue when B < 1 or the grid would be too large.
hipError_t exact_predict(const ExactArgs& a, int B, bool f32, hipStream_t st);

// The rapid method's interpolated covariance of one site at arbitrary points (eq. weights):
// out[j] = sum_{m < M} W[m] k(|p_j - g_m|), g_m the site's neighbour nodes (anchor (i0, j0),
// offsets (ox, oy) in {-L+1..L}^2, ox-major), W its M weights.  FP64.
hipError_t kernel_approx_at(const GridDev& g, const MaternDev& mt, int i0, int j0, const double* W,
                            const double* pts, int npts, double* out, hipStream_t st);

}  // namespace krig
