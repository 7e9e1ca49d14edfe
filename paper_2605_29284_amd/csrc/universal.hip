// Universal kriging (Section 3: the GLS trend estimate and the coefficients of the
// spatial part, eqs. findbeta, findc and predictionf).  The spatial part goes through
// the plan's solve and rapid convolution; these kernels form the small GLS system,
// solve it, correct the coefficients and add the trend on the grid.
#include "universal.h"

#include <math.h>

namespace krig {

// one block per entry of G, 256 threads: strided partial sums, then a fixed LDS tree
__global__ void __launch_bounds__(256) k_uk_gram(const double* __restrict__ Xs, const double* __restrict__ VX,
                                                 const double* __restrict__ U, int n, int np, double* __restrict__ G) {
  __shared__ double red[256];
  const int r = blockIdx.x, l = blockIdx.y;
  const double* a = Xs + (int64_t)r * n;
  const double* b = l < np ? VX + (int64_t)l * n : U + (int64_t)(l - np) * n;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += a[i] * b[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) G[(int64_t)r * gridDim.y + l] = red[0];  // row pitch np + B
}

hipError_t uk_gram(const double* Xs, const double* VX, const double* U, int n, int np, int B, double* G,
                   hipStream_t st) {
  if (np < 1 || np > UK_MAX || B < 1 || B > 65535 - UK_MAX) return hipErrorInvalidValue;
  k_uk_gram<<<dim3(np, np + B), 256, 0, st>>>(Xs, VX, U, n, np, G);
  return hipGetLastError();
}

// one block: thread 0 factors A = L L^T (lower) in LDS, then every thread solves its
// right-hand sides by forward and back substitution
__global__ void __launch_bounds__(256) k_uk_solve(const double* __restrict__ G, int np, int B,
                                                  double* __restrict__ beta) {
  __shared__ double Lf[UK_MAX][UK_MAX];
  __shared__ int ok;
  const int ld = np + B;
  if (threadIdx.x == 0) {
    ok = 1;
    for (int i = 0; i < np; ++i)
      for (int j = 0; j <= i; ++j) Lf[i][j] = G[(int64_t)i * ld + j];
    for (int j = 0; j < np && ok; ++j) {
      // a pivot below 1e-8 of its diagonal entry (covariate j reproduced by the earlier ones
      // to about four digits in the M^{-1} inner product) counts as dependent: the sign of a
      // rounding residue must not decide it
      const double d0 = Lf[j][j];
      double d = d0;
      for (int k = 0; k < j; ++k) d -= Lf[j][k] * Lf[j][k];
      if (!(d > 1e-8 * d0)) {
        ok = 0;
        break;
      }
      d = sqrt(d);
      Lf[j][j] = d;
      for (int i = j + 1; i < np; ++i) {
        double v = Lf[i][j];
        for (int k = 0; k < j; ++k) v -= Lf[i][k] * Lf[j][k];
        Lf[i][j] = v / d;
      }
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    double x[UK_MAX];
    if (!ok) {
      for (int k = 0; k < np; ++k) beta[(int64_t)b * np + k] = NAN;
      continue;
    }
    for (int i = 0; i < np; ++i) {  // L y = h
      double v = G[(int64_t)i * ld + np + b];
      for (int k = 0; k < i; ++k) v -= Lf[i][k] * x[k];
      x[i] = v / Lf[i][i];
    }
    for (int i = np - 1; i >= 0; --i) {  // L^T beta = y
      double v = x[i];
      for (int k = i + 1; k < np; ++k) v -= Lf[k][i] * x[k];
      x[i] = v / Lf[i][i];
    }
    for (int k = 0; k < np; ++k) beta[(int64_t)b * np + k] = x[k];
  }
}

hipError_t uk_solve(const double* G, int np, int B, double* beta, hipStream_t st) {
  if (np < 1 || np > UK_MAX || B < 1) return hipErrorInvalidValue;
  k_uk_solve<<<1, 256, 0, st>>>(G, np, B, beta);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_uk_resid(double* __restrict__ U, const double* __restrict__ VX,
                                                  const double* __restrict__ beta, int n, int np, int64_t tot) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int64_t b = idx / n, i = idx % n;
  double v = U[idx];
  for (int k = 0; k < np; ++k) v -= VX[(int64_t)k * n + i] * beta[b * np + k];
  U[idx] = v;
}

hipError_t uk_resid(double* U, const double* VX, const double* beta, int n, int np, int B, hipStream_t st) {
  const int64_t tot = (int64_t)n * B;
  if (tot <= 0) return hipSuccess;
  k_uk_resid<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(U, VX, beta, n, np, tot);
  return hipGetLastError();
}

template <typename TS>
__global__ void __launch_bounds__(256) k_uk_trend(TS* __restrict__ yhat, const double* __restrict__ Xg,
                                                  const double* __restrict__ beta, int64_t npix, int np, int64_t tot) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int64_t b = idx / npix, q = idx % npix;
  double v = (double)yhat[idx];
  for (int k = 0; k < np; ++k) v += Xg[(int64_t)k * npix + q] * beta[b * np + k];
  yhat[idx] = (TS)v;
}

hipError_t uk_trend(void* yhat, bool f32, const double* Xg, const double* beta, int64_t npix, int np, int B,
                    hipStream_t st) {
  const int64_t tot = npix * B;
  if (tot <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((tot + 255) / 256);
  if (f32)
    k_uk_trend<float><<<grid, 256, 0, st>>>(reinterpret_cast<float*>(yhat), Xg, beta, npix, np, tot);
  else
    k_uk_trend<double><<<grid, 256, 0, st>>>(reinterpret_cast<double*>(yhat), Xg, beta, npix, np, tot);
  return hipGetLastError();
}

}  // namespace krig
