// Universal kriging: the GLS trend of eqs. findbeta / findc / predictionf (GPU helpers).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace krig {

constexpr int UK_MAX = 16;  // covariates

// G[r][l] = sum_i Xs[r][i] R_l[i], r < np, l < np + B, where R_l = VX[l] (l < np) or
// U[l - np]; all rows have n entries.  Fixed-order reduction.
hipError_t uk_gram(const double* Xs, const double* VX, const double* U, int n, int np, int B, double* G,
                   hipStream_t st);
// beta[b][k] from G = [A | H] (A = X^T M^{-1} X, H = X^T M^{-1} z): A beta_b = H[:, b];
// NaN for every b when A is not numerically positive definite.
hipError_t uk_solve(const double* G, int np, int B, double* beta, hipStream_t st);
// U[b][i] -= sum_k VX[k][i] beta[b][k]  (c = M^{-1} z - M^{-1} X beta)
hipError_t uk_resid(double* U, const double* VX, const double* beta, int n, int np, int B, hipStream_t st);
// yhat[b][q] += sum_k Xg[k][q] beta[b][k], q < npix (FP64 sum, one rounding)
hipError_t uk_trend(void* yhat, bool f32, const double* Xg, const double* beta, int64_t npix, int np, int B,
                    hipStream_t st);

}  // namespace krig
