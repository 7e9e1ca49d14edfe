// Exact kriging predictions (eq. predictionh), the O(N n) product the rapid method replaces.
// EX_PP evaluation points per thread and up to EX_FB fields per block row: tiles of sites and
// their coefficients are staged in LDS (every lane reads the same entry, a broadcast), each
// covariance k(|p - s_i|) is evaluated once per point and site and used for all the row's
// fields.  The sum runs over the sites in index order in FP64.
#include "exact.h"

#include <math.h>

namespace krig {

namespace {
constexpr int EX_FB = 16;     // fields per block row
constexpr int EX_TILE = 256;  // sites per LDS tile (= threads per block)
constexpr int EX_PP = 1;      // points per thread
}  // namespace

template <typename TS, bool GRID>
__device__ inline void exact_point(const ExactArgs& a, int j, double& px, double& py) {
  if constexpr (GRID) {
    px = a.g.x0 + (double)(j / a.g.m2) * a.g.dx;
    py = a.g.y0 + (double)(j % a.g.m2) * a.g.dy;
  } else {
    px = a.pts[2 * (int64_t)j];
    py = a.pts[2 * (int64_t)j + 1];
  }
}

// Each thread takes EX_PP points (j, j + EX_TILE, ... of its block's span); a site's EX_FB
// coefficients are contiguous in LDS and read as 16-byte broadcasts.  One point per thread
// measured fastest on the paper-sized grid (two per thread halve the LDS reads per pair but
// also the number of blocks, and 350 x 350 points then fill fewer than one block per CU).
template <typename TS, bool GRID>
__global__ void __launch_bounds__(EX_TILE) k_exact(ExactArgs a, int B, int npoints) {
  __shared__ double sx[EX_TILE], sy[EX_TILE];
  __shared__ __align__(16) double sa[EX_TILE][EX_FB];
  const int f0 = blockIdx.y * EX_FB;
  const int nf = min(EX_FB, B - f0);
  int jp[EX_PP];
  double px[EX_PP], py[EX_PP];
#pragma unroll
  for (int h = 0; h < EX_PP; ++h) {
    jp[h] = blockIdx.x * (EX_PP * EX_TILE) + h * EX_TILE + threadIdx.x;
    px[h] = py[h] = 0.0;
    if (jp[h] < npoints) exact_point<TS, GRID>(a, jp[h], px[h], py[h]);
  }
  double acc[EX_PP][EX_FB];
#pragma unroll
  for (int h = 0; h < EX_PP; ++h)
#pragma unroll
    for (int f = 0; f < EX_FB; ++f) acc[h][f] = 0.0;
  for (int t0 = 0; t0 < a.n; t0 += EX_TILE) {
    const int cnt = min(EX_TILE, a.n - t0);
    __syncthreads();  // the previous tile has been used by every thread
    if ((int)threadIdx.x < cnt) {
      const int i = t0 + threadIdx.x;
      sx[threadIdx.x] = a.sites[2 * (int64_t)i];
      sy[threadIdx.x] = a.sites[2 * (int64_t)i + 1];
#pragma unroll
      for (int f = 0; f < EX_FB; ++f) sa[threadIdx.x][f] = f < nf ? a.alpha[(int64_t)(f0 + f) * a.alpha_fs + i] : 0.0;
    }
    __syncthreads();
    for (int u = 0; u < cnt; ++u) {
      double kv[EX_PP];
#pragma unroll
      for (int h = 0; h < EX_PP; ++h) {
        const double ddx = px[h] - sx[u], ddy = py[h] - sy[u];
        kv[h] = matern_cov(sqrt(ddx * ddx + ddy * ddy), a.mt);
      }
#pragma unroll
      for (int f = 0; f < EX_FB; ++f) {
        const double c = sa[u][f];
#pragma unroll
        for (int h = 0; h < EX_PP; ++h) acc[h][f] += kv[h] * c;
      }
    }
  }
  TS* o = reinterpret_cast<TS*>(a.out);
#pragma unroll
  for (int h = 0; h < EX_PP; ++h) {
    if (jp[h] >= npoints) continue;
#pragma unroll
    for (int f = 0; f < EX_FB; ++f)
      if (f < nf) o[(int64_t)(f0 + f) * a.out_fs + jp[h]] = (TS)acc[h][f];
  }
}

hipError_t exact_predict(const ExactArgs& a, int B, bool f32, hipStream_t st) {
  const bool grid = a.pts == nullptr;
  const int64_t np = grid ? (int64_t)a.g.m1 * a.g.m2 : a.npts;
  if (B < 1 || np < 0 || np > (int64_t)1 << 30 || (B + EX_FB - 1) / EX_FB > 65535) return hipErrorInvalidValue;
  if (np == 0) return hipSuccess;
  const dim3 blocks((unsigned)((np + EX_PP * EX_TILE - 1) / (EX_PP * EX_TILE)), (unsigned)((B + EX_FB - 1) / EX_FB));
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

__global__ void __launch_bounds__(256) k_kernel_approx(GridDev g, MaternDev mt, int i0, int j0,
                                                       const double* __restrict__ W, const double* __restrict__ pts,
                                                       int npts, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= npts) return;
  const double px = pts[2 * (int64_t)j], py = pts[2 * (int64_t)j + 1];
  const int L2 = 2 * g.L;
  double s = 0.0;
  for (int m = 0; m < g.M; ++m) {
    const int ox = m / L2 - g.L + 1, oy = m % L2 - g.L + 1;
    const double ddx = px - (g.x0 + (double)(i0 + ox) * g.dx), ddy = py - (g.y0 + (double)(j0 + oy) * g.dy);
    s += W[m] * matern_cov(sqrt(ddx * ddx + ddy * ddy), mt);
  }
  out[j] = s;
}

hipError_t kernel_approx_at(const GridDev& g, const MaternDev& mt, int i0, int j0, const double* W,
                            const double* pts, int npts, double* out, hipStream_t st) {
  if (npts <= 0) return npts == 0 ? hipSuccess : hipErrorInvalidValue;
  hipLaunchKernelGGL(k_kernel_approx, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, g, mt, i0, j0, W, pts,
                     npts, out);
  return hipGetLastError();
}

}  // namespace krig
