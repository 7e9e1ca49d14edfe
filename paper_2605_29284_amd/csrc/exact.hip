// Exact kriging predictions (eq. predictionh), the O(N n) product the rapid method replaces.
// One thread per evaluation point and up to EX_FB fields per block row: tiles of sites and
// their coefficients are staged in LDS (every lane reads the same entry, a broadcast), each
// covariance k(|p - s_i|) is evaluated once per point and site and used for all the row's
// fields.  The sum runs over the sites in index order in FP64.
#include "exact.h"

#include <math.h>

namespace krig {

namespace {
constexpr int EX_FB = 16;     // fields per block row
constexpr int EX_TILE = 256;  // sites per LDS tile (= threads per block)
}  // namespace

template <typename TS, bool GRID>
__global__ void __launch_bounds__(EX_TILE) k_exact(ExactArgs a, int B, int npoints) {
  __shared__ double sx[EX_TILE], sy[EX_TILE], sa[EX_FB][EX_TILE];
  const int j = blockIdx.x * EX_TILE + threadIdx.x;
  const int f0 = blockIdx.y * EX_FB;
  const int nf = min(EX_FB, B - f0);
  const bool ok = j < npoints;
  double px = 0.0, py = 0.0;
  if (ok) {
    if constexpr (GRID) {
      px = a.g.x0 + (double)(j / a.g.m2) * a.g.dx;
      py = a.g.y0 + (double)(j % a.g.m2) * a.g.dy;
    } else {
      px = a.pts[2 * (int64_t)j];
      py = a.pts[2 * (int64_t)j + 1];
    }
  }
  double acc[EX_FB];
#pragma unroll
  for (int f = 0; f < EX_FB; ++f) acc[f] = 0.0;
  for (int t0 = 0; t0 < a.n; t0 += EX_TILE) {
    const int cnt = min(EX_TILE, a.n - t0);
    __syncthreads();  // the previous tile has been used by every thread
    if ((int)threadIdx.x < cnt) {
      const int i = t0 + threadIdx.x;
      sx[threadIdx.x] = a.sites[2 * (int64_t)i];
      sy[threadIdx.x] = a.sites[2 * (int64_t)i + 1];
#pragma unroll
      for (int f = 0; f < EX_FB; ++f) sa[f][threadIdx.x] = f < nf ? a.alpha[(int64_t)(f0 + f) * a.alpha_fs + i] : 0.0;
    }
    __syncthreads();
    for (int u = 0; u < cnt; ++u) {
      const double ddx = px - sx[u], ddy = py - sy[u];
      const double kv = matern_cov(sqrt(ddx * ddx + ddy * ddy), a.mt);
#pragma unroll
      for (int f = 0; f < EX_FB; ++f) acc[f] += kv * sa[f][u];
    }
  }
  if (!ok) return;
  TS* o = reinterpret_cast<TS*>(a.out);
#pragma unroll
  for (int f = 0; f < EX_FB; ++f)
    if (f < nf) o[(int64_t)(f0 + f) * a.out_fs + j] = (TS)acc[f];
}

hipError_t exact_predict(const ExactArgs& a, int B, bool f32, hipStream_t st) {
  const bool grid = a.pts == nullptr;
  const int64_t np = grid ? (int64_t)a.g.m1 * a.g.m2 : a.npts;
  if (B < 1 || np < 0 || np > (int64_t)1 << 30 || (B + EX_FB - 1) / EX_FB > 65535) return hipErrorInvalidValue;
  if (np == 0) return hipSuccess;
  const dim3 blocks((unsigned)((np + EX_TILE - 1) / EX_TILE), (unsigned)((B + EX_FB - 1) / EX_FB));
  const int npi = (int)np;
  if (grid) {
    if (f32)
      hipLaunchKernelGGL((k_exact<float, true>), blocks, dim3(EX_TILE), 0, st, a, B, npi);
    else
      hipLaunchKernelGGL((k_exact<double, true>), blocks, dim3(EX_TILE), 0, st, a, B, npi);
  } else {
    if (f32)
      hipLaunchKernelGGL((k_exact<float, false>), blocks, dim3(EX_TILE), 0, st, a, B, npi);
    else
      hipLaunchKernelGGL((k_exact<double, false>), blocks, dim3(EX_TILE), 0, st, a, B, npi);
  }
  return hipGetLastError();
}

}  // namespace krig
