// Off-grid predictions from the mesh prediction by local Lagrange interpolation (GPU).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace krig {

struct InterpArgs {
  const void* yhat;     // mesh prediction [B][m1][m2] (float or double), field pitch yhat_fs
  int64_t yhat_fs;
  int m1, m2;
  double x0, y0, dx, dy;
  const double* pts;    // [npts][2] FP64
  int npts;
  void* out;            // [B][npts] (same type as yhat), field pitch out_fs
  int64_t out_fs;
};

// out[b][j] = sum_{p,c < q} l_p(t_j) l_c(u_j) yhat[b][sx + p][sy + c]; q in [2, 8], q <= m1, m2.
// NaN for points outside the grid's bounding box.  hipErrorInvalidValue on a bad q or B.
hipError_t interp_points(const InterpArgs& a, int B, int q, bool f32, hipStream_t st);

}  // namespace krig
