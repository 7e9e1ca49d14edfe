// FP64 dense linear algebra on the GPU: the kriging system M = K + tau^2 I of
// eq. (findc), factored by a blocked right-looking Cholesky whose panel solves and
// trailing updates are FP64 MFMA GEMMs, and the explicit inverse Cholesky factor
// L^{-1} used to apply M^{-1} = L^{-T} L^{-1} to many right-hand sides at once.
#include "dense.h"

#include <math.h>

#include "matern_dev.h"

namespace krig {

typedef double double4_t __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------------
// GEMM: C = alpha * op(A) * op(B) + beta * C  (row-major, FP64, MFMA 16x16x4)
// Block tile 64 x 64, four waves each owning a 32 x 32 quadrant (2 x 2 MFMA tiles),
// K staged through two LDS buffers 16 at a time (register prefetch of the next chunk).
// LOWER restricts the launch to tiles with tile_col <= tile_row (symmetric rank-k updates).
// MFMA operand layout (v_mfma_f64_16x16x4f64): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; result register r of lane l is D[l/16 + 4*r][l%16] (FP64 form: rows
// interleave across the four lane groups, unlike the FP32 16x16 forms).
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_gemm_f64(GemmArgs g) {
  // two LDS buffers: chunk t is staged into buffer t&1 while the previous chunk's MFMAs run,
  // and the next chunk's global loads are in flight in registers during chunk t's MFMAs
  __shared__ double As[2][16][64 + 1];   // [buf][k][m]
  __shared__ double Bs[2][16][64 + 1];   // [buf][k][n]
  const int tm = blockIdx.y, tn = blockIdx.x;
  if (g.lower && tn > tm) return;
  const int m0 = tm * 64 + g.m_off, n0 = tn * 64 + g.n_off;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  double4_t acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};

  // element e = tid + 256 q (q < 4) of a 64 x 16 chunk: its (m, k) and (n, k) positions
  int am[4], ak[4], bn[4], bk[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + 256 * q;
    if (g.transA) { am[q] = e % 64; ak[q] = e / 64; } else { ak[q] = e % 16; am[q] = e / 16; }
    if (g.transB) { bk[q] = e % 16; bn[q] = e / 16; } else { bn[q] = e % 64; bk[q] = e / 64; }
  }
  double ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gm = m0 + am[q], gka = k0 + ak[q];
      ra[q] = 0.0;
      if (gm < g.M_end && gka < g.K)
        ra[q] = g.transA ? g.A[(int64_t)gka * g.lda + gm] : g.A[(int64_t)gm * g.lda + gka];
      const int gn = n0 + bn[q], gkb = k0 + bk[q];
      rb[q] = 0.0;
      if (gn < g.N_end && gkb < g.K)
        rb[q] = g.transB ? g.B[(int64_t)gn * g.ldb + gkb] : g.B[(int64_t)gkb * g.ldb + gn];
    }
  };
  fetch(0);
  int buf = 0;
  for (int k0 = 0; k0 < g.K; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      As[buf][ak[q]][am[q]] = ra[q];
      Bs[buf][bk[q]][bn[q]] = rb[q];
    }
    __syncthreads();  // chunk visible; every wave is past the MFMAs that last read this buffer's twin
    if (k0 + 16 < g.K) fetch(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int kq = kk + (lane >> 4);
      double a0 = As[buf][kq][wm + (lane & 15)];
      double a1 = As[buf][kq][wm + 16 + (lane & 15)];
      double b0 = Bs[buf][kq][wn + (lane & 15)];
      double b1 = Bs[buf][kq][wn + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    buf ^= 1;
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
        const int gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < g.M_end && gn < g.N_end) {
          if (g.lower && gn > gm) continue;
          double* c = g.C + (int64_t)gm * g.ldc + gn;
          const double v = g.alpha * acc[i][j][r];
          *c = (g.beta == 0.0) ? v : v + g.beta * *c;
        }
      }
}

hipError_t gemm_f64(const GemmArgs& g, hipStream_t st) {
  const int M = g.M_end - g.m_off, N = g.N_end - g.n_off;
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL(k_gemm_f64, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// assembly of M = K + tau^2 I (full square, row-major)
// ------------------------------------------------------------------------------------
__global__ void k_assemble_kt(const double* __restrict__ sites, int n, MaternDev mt, double* __restrict__ Kt,
                              int64_t ld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  const double hx = sites[2 * i] - sites[2 * j];
  const double hy = sites[2 * i + 1] - sites[2 * j + 1];
  double v = matern_cov(sqrt(hx * hx + hy * hy), mt);
  if (i == j) v += mt.tau2;
  Kt[(int64_t)i * ld + j] = v;
}

hipError_t assemble_kt(const double* d_sites, int n, const MaternDev& mt, double* Kt, int64_t ld,
                       hipStream_t st) {
  const int64_t tot = (int64_t)n * n;
  hipLaunchKernelGGL(k_assemble_kt, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, d_sites, n, mt, Kt,
                     ld);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// diagonal block: Cholesky of a 64 x 64 tile (in place, lower) and its inverse.
// Entries past the matrix edge act as the identity.  A non-positive pivot stores
// (global row + 1) into *status (first failure wins) and the tile is left as is.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_potrf_diag(double* A, int64_t lda, int n, int k0, double* Dinv,
                                                    int* status) {
  __shared__ double a[64][65];
  __shared__ double dinv[64];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int nb = min(64, n - k0);
  if (tid == 0) bad = 0;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e / 64, j = e % 64;
    double v = 0.0;
    if (i < nb && j < nb) v = (j <= i) ? A[(int64_t)(k0 + i) * lda + k0 + j] : 0.0;
    else if (i == j) v = 1.0;
    a[i][j] = v;
  }
  __syncthreads();
  // right-looking column sweep; thread (ti, tj) of a 16 x 16 grid owns rows 4ti..4ti+3 and
  // columns 4tj..4tj+3 of the trailing update (lower triangle only)
  const int ti = tid >> 4, tj = tid & 15;
  for (int j = 0; j < 64; ++j) {
    if (tid == 0) {
      const double d = a[j][j];
      if (!(d > 0.0)) {
        if (!bad) {
          bad = 1;
          atomicCAS(status, 0, k0 + j + 1);
        }
        a[j][j] = 1.0;
      } else {
        a[j][j] = sqrt(d);
      }
    }
    __syncthreads();
    if (tid > j && tid < 64) a[tid][j] /= a[j][j];
    __syncthreads();
    if (4 * ti + 3 > j && 4 * tj + 3 > j && tj <= ti) {
      double li[4], lc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        li[u] = a[4 * ti + u][j];
        lc[u] = a[4 * tj + u][j];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 4 * ti + u, c = 4 * tj + v;
          if (i > j && c > j && c <= i) a[i][c] -= li[u] * lc[v];
        }
    }
    __syncthreads();
  }
  // the factor back to A
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e / 64, j = e % 64;
    if (i < nb && j < nb) A[(int64_t)(k0 + i) * lda + k0 + j] = (j <= i) ? a[i][j] : 0.0;
  }
  // inverse of the lower-triangular tile by forward substitution, one column per thread:
  // entry (i, j), i > j, of the inverse is kept at a[j][i] (the unused upper triangle, row j
  // belongs to thread j alone) and the diagonal in dinv; the factor itself stays in the
  // lower triangle, which is only read from here on
  if (tid < 64) {
    const int j = tid;
    const double djj = 1.0 / a[j][j];
    dinv[j] = djj;
    for (int i = j + 1; i < 64; ++i) {
      double s = a[i][j] * djj;
      for (int k = j + 1; k < i; ++k) s += a[i][k] * a[j][k];
      a[j][i] = -s / a[i][i];
    }
  }
  __syncthreads();
  // Dinv row-major 64 x 64 (lower), coalesced
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e / 64, j = e % 64;
    Dinv[e] = i > j ? a[j][i] : (i == j ? dinv[i] : 0.0);
  }
}

// zero the strict upper triangle of an n x n row-major matrix
__global__ void k_zero_upper(double* A, int64_t lda, int n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  if (j > i) A[(int64_t)i * lda + j] = 0.0;
}

constexpr int CHOL_GROUP = 4;  // 64-wide blocks per outer panel of the factorisations

// Blocked Cholesky of the n x n matrix A (lower, in place) plus the inverse factor
// Linv = L^{-1} (lower, n x n).  work: 64 x n doubles.  Dinv: nblk * 64 * 64.
hipError_t cholesky_and_inverse(double* A, int64_t lda, int n, double* Linv, double* Dinv, double* work,
                                int* d_status, hipStream_t st) {
  const int nblk = (n + 63) / 64;
  hipError_t e;
  for (int kb = 0; kb < nblk; ++kb) {
    const int k0 = kb * 64;
    const int nb = min(64, n - k0);
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, st, A, lda, n, k0, Dinv + (int64_t)kb * 4096,
                       d_status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (k0 + nb >= n) break;
    // panel: L21 = A21 * Dinv^T  (rows k0+nb .. n-1, cols k0 .. k0+nb-1), via work
    {
      const int rows = n - k0 - nb;
      GemmArgs g{};
      g.A = A + (int64_t)(k0 + nb) * lda + k0; g.lda = lda; g.transA = 0;
      g.B = Dinv + (int64_t)kb * 4096; g.ldb = 64; g.transB = 1;
      g.C = work; g.ldc = 64;
      g.m_off = 0; g.M_end = rows; g.n_off = 0; g.N_end = nb; g.K = nb;
      g.alpha = 1.0; g.beta = 0.0; g.lower = 0;
      if ((e = gemm_f64(g, st)) != hipSuccess) return e;
      // copy back into A
      if ((e = copy_rows(work, 64, A + (int64_t)(k0 + nb) * lda + k0, lda, rows, nb, st)) != hipSuccess) return e;
    }
    // trailing update A22 -= L21 L21^T (lower tiles).  Blocks go in groups of CHOL_GROUP
    // (outer panels of 64 CHOL_GROUP columns): within a group a block updates only the
    // group's remaining columns (K = 64); the group's last block updates everything to
    // the right at once from all the group's columns (K = 64 CHOL_GROUP), which divides
    // the trailing matrix's read-modify-write traffic by CHOL_GROUP.
    {
      const int rows = n - k0 - nb;
      const int g0 = (kb - kb % CHOL_GROUP) * 64;  // first column of the group
      const bool last = kb % CHOL_GROUP == CHOL_GROUP - 1;
      const int kc = last ? g0 : k0;               // first column of the update's K range
      GemmArgs g{};
      g.A = A + (int64_t)(k0 + nb) * lda + kc; g.lda = lda; g.transA = 0;
      g.B = A + (int64_t)(k0 + nb) * lda + kc; g.ldb = lda; g.transB = 1;
      g.C = A + (int64_t)(k0 + nb) * lda + (k0 + nb); g.ldc = lda;
      g.m_off = 0; g.M_end = rows; g.n_off = 0;
      g.N_end = last ? rows : min(g0 + 64 * CHOL_GROUP - (k0 + nb), rows);
      g.K = k0 + nb - kc;
      g.alpha = -1.0; g.beta = 1.0; g.lower = 1;
      if ((e = gemm_f64(g, st)) != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_zero_upper, dim3((unsigned)(((int64_t)n * n + 255) / 256)), dim3(256), 0, st, A, lda, n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (!Linv) return hipSuccess;
  // Linv by block forward substitution on L X = I.  X (in Linv) first accumulates
  // R[i][j] = sum_{j<=k<i} L_ik X_kj; block row i is then X[i][:i] = -Dinv_i R[i][:i],
  // X[i][i] = Dinv_i, and R of the rows below is updated with L[:, i] X[i][:i+1].
  if ((e = fill_f64(Linv, (int64_t)n * lda, 0.0, st)) != hipSuccess) return e;
  for (int ib = 0; ib < nblk; ++ib) {
    const int i0 = ib * 64;
    const int nb = min(64, n - i0);
    if (ib > 0) {
      // X[i][0:i0] = -Dinv_i R[i][0:i0]   (via work: 64 x i0)
      GemmArgs g{};
      g.A = Dinv + (int64_t)ib * 4096; g.lda = 64; g.transA = 0;
      g.B = Linv + (int64_t)i0 * lda; g.ldb = lda; g.transB = 0;
      g.C = work; g.ldc = n;
      g.m_off = 0; g.M_end = nb; g.n_off = 0; g.N_end = i0; g.K = nb;
      g.alpha = -1.0; g.beta = 0.0; g.lower = 0;
      if ((e = gemm_f64(g, st)) != hipSuccess) return e;
      if ((e = copy_rows(work, n, Linv + (int64_t)i0 * lda, lda, nb, i0, st)) != hipSuccess) return e;
    }
    // diagonal block
    if ((e = copy_rows(Dinv + (int64_t)ib * 4096, 64, Linv + (int64_t)i0 * lda + i0, lda, nb, nb, st)) !=
        hipSuccess)
      return e;
    if (i0 + nb >= n) break;
    // R[i0+nb:, 0:i0+nb] += L[i0+nb:, i0:i0+nb] X[i0:i0+nb, 0:i0+nb], with the block rows in
    // groups as in the factorisation: within a group a block row updates only the group's
    // remaining block rows (K = 64); the group's last updates all rows below from the whole
    // group (K = 64 CHOL_GROUP; X of an earlier block row is zero in later ones' columns)
    const int g0 = (ib - ib % CHOL_GROUP) * 64;
    const bool last = ib % CHOL_GROUP == CHOL_GROUP - 1;
    const int kc = last ? g0 : i0;
    GemmArgs g{};
    g.A = A + (int64_t)(i0 + nb) * lda + kc; g.lda = lda; g.transA = 0;
    g.B = Linv + (int64_t)kc * lda; g.ldb = lda; g.transB = 0;
    g.C = Linv + (int64_t)(i0 + nb) * lda; g.ldc = lda;
    g.m_off = 0; g.M_end = last ? n - i0 - nb : min(g0 + 64 * CHOL_GROUP - (i0 + nb), n - i0 - nb);
    g.n_off = 0; g.N_end = i0 + nb;
    g.K = i0 + nb - kc;
    g.alpha = 1.0; g.beta = 1.0; g.lower = 0;
    if ((e = gemm_f64(g, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

__global__ void k_fill_f64(double* p, int64_t cnt, double v) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < cnt) p[idx] = v;
}

hipError_t fill_f64(double* p, int64_t cnt, double v, hipStream_t st) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, p, cnt, v);
  return hipGetLastError();
}

__global__ void k_copy_rows(const double* __restrict__ src, int64_t lds_, double* __restrict__ dst, int64_t ldd,
                            int nr, int nc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nr * nc) return;
  const int i = (int)(idx / nc), j = (int)(idx % nc);
  dst[(int64_t)i * ldd + j] = src[(int64_t)i * lds_ + j];
}

hipError_t copy_rows(const double* src, int64_t ld_src, double* dst, int64_t ld_dst, int nr, int nc,
                     hipStream_t st) {
  const int64_t tot = (int64_t)nr * nc;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, src, ld_src, dst,
                     ld_dst, nr, nc);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// transpose of an n x n row-major matrix into dst (pitch ldd), through 32 x 32 LDS tiles
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_transpose_f64(const double* __restrict__ src, int64_t lds_,
                                                       double* __restrict__ dst, int64_t ldd, int n) {
  __shared__ double t[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    t[k][tx] = (r < n && c < n) ? src[(int64_t)r * lds_ + c] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int r = c0 + k, c = r0 + tx;
    if (r < n && c < n) dst[(int64_t)r * ldd + c] = t[tx][k];
  }
}

hipError_t transpose_f64(const double* src, int64_t ld_src, double* dst, int64_t ld_dst, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  dim3 grid((n + 31) / 32, (n + 31) / 32);
  hipLaunchKernelGGL(k_transpose_f64, grid, dim3(256), 0, st, src, ld_src, dst, ld_dst, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// triangular product with an explicit triangular factor T (row-major, pitch ldt,
// zeros outside the triangle and in the pitch padding):
//   upper = 0:  out[b][i] = sum_{k <= i} T[i][k] in[b][k]      (T = L^{-1})
//   upper = 1:  out[b][i] = sum_{k >= i} T[i][k] in[b][k]      (T = L^{-T})
// One workgroup of TRI_NW waves owns an output tile: 16 rows (row tile t) x 16 fields
// (group z), over the tile's chunks of 16 columns inside the triangle.  Wave w takes chunks
// w, w + TRI_NW, ... (the waves read neighbouring row segments together), KS chunks in
// flight at a time (six in a plain launch: 96 chunks per round trip covers n <= 1536 in one;
// five in the persistent form, whose loop holds more registers).  KS does not change the
// order in which a wave adds its chunks, so both forms give the same bits.  Per chunk, lane (r = l%16, g = l/16) loads T[16t+r][16c + 4g .. +3] as
// one 32-byte vector (whole 128-byte row segments per wave) and in[16z+r][same k]; four MFMA
// 16x16x4 steps take element s of each, so the K order inside a chunk is permuted identically
// for both operands.  The waves' partial tiles are added through LDS in wave order: one launch
// per product, no partials in device memory, bitwise repeatable results.
//
// Short products (few 16 x 16 tiles for the compute units) take 8-row x 8-field tiles instead
// (TRI_FORM8).  A workgroup's time there is its heaviest tile streaming its K range through one
// compute unit, (rows + fields) x K x 8 bytes; the 8 x 8 form halves that.  Its chunks are 32
// columns wide and the MFMA's 16 x 16 operands hold two K ranges side by side: operand rows and
// columns 0-7 take columns 32c .. 32c+15 of the tile's 8 fields and 8 rows, rows and columns 8-15
// columns 32c+16 .. 32c+31 of the same ones.  The two diagonal 8 x 8 blocks of the result are
// the two ranges' partial sums (the off-diagonal blocks mix ranges and are dropped), added with
// the waves' partials in a fixed order.  The heaviest tiles are dispatched first.  Four 32-column
// chunks in flight per wave cover rows of up to 2048 columns in one memory round trip.
// ------------------------------------------------------------------------------------
constexpr int TRI_NW = 16;  // waves per tile

// VEC: in_fs is a multiple of 4 and in 32-byte aligned, so a lane's four input values
// are one 32-byte load (values past n are masked to zero).
template <int UPPER, bool VEC, int KS>
__device__ __forceinline__ void tri_tile_body(const double* __restrict__ T, int64_t ldt, int n,
                                              const double* __restrict__ in, int64_t in_fs, int B,
                                              double* __restrict__ out, int64_t out_fs, int t, int z,
                                              double (*red)[256]) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
  const int i0 = 16 * t, f0 = 16 * z;
  const int nch = (n + 15) / 16;
  const int cbeg = UPPER ? t : 0, cend = UPPER ? nch : t + 1;
  const bool rok = i0 + r < n, fok = f0 + r < B;
  const double* trow = T + (int64_t)(rok ? i0 + r : 0) * ldt;
  const double* irow = in + (int64_t)(fok ? f0 + r : 0) * in_fs;
  double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
  for (int cb = cbeg + w; cb < cend; cb += TRI_NW * KS) {
    double4_t x[KS];
    double a[KS][4];
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int c = cb + u * TRI_NW;
      const int k = 16 * c + 4 * g;
      x[u] = (double4_t){0.0, 0.0, 0.0, 0.0};
      if (rok && c < cend) x[u] = *reinterpret_cast<const double4_t*>(trow + k);
      if constexpr (VEC) {
        double4_t av = (double4_t){0.0, 0.0, 0.0, 0.0};
        if (fok && c < cend && k < n) av = *reinterpret_cast<const double4_t*>(irow + k);
#pragma unroll
        for (int s = 0; s < 4; ++s) a[u][s] = k + s < n ? av[s] : 0.0;
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) a[u][s] = (fok && c < cend && k + s < n) ? irow[k + s] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < KS; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][s], x[u][s], acc, 0, 0, 0);
  }
  // element e = 64 j + lane of a partial tile is MFMA result register j of lane `lane`:
  // field f0 + lane/16 + 4 j, row i0 + lane%16
#pragma unroll
  for (int j = 0; j < 4; ++j) red[w][j * 64 + lane] = acc[j];
  __syncthreads();
  if (tid < 256) {
    double s = 0.0;
#pragma unroll
    for (int v = 0; v < TRI_NW; ++v) s += red[v][tid];
    const int f = f0 + ((tid & 63) >> 4) + 4 * (tid >> 6), i = i0 + (tid & 15);
    if (f < B && i < n) out[(int64_t)f * out_fs + i] = s;
  }
}

// the 8-row x 8-field form: rows 8t .. 8t+7, fields 8z .. 8z+7, chunks of 32 columns
template <int UPPER, bool VEC, int KS>
__device__ __forceinline__ void tri_tile8_body(const double* __restrict__ T, int64_t ldt, int n,
                                               const double* __restrict__ in, int64_t in_fs, int B,
                                               double* __restrict__ out, int64_t out_fs, int t, int z,
                                               double (*red)[256]) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
  const int rr = r & 7, h = r >> 3;  // row / field within the tile, K range of the chunk
  const int i0 = 8 * t, f0 = 8 * z;
  const int cbeg = UPPER ? i0 / 32 : 0, cend = UPPER ? (n + 31) / 32 : (i0 + 39) / 32;
  const bool rok = i0 + rr < n, fok = f0 + rr < B;
  const double* trow = T + (int64_t)(rok ? i0 + rr : 0) * ldt;
  const double* irow = in + (int64_t)(fok ? f0 + rr : 0) * in_fs;
  double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
  for (int cb = cbeg + w; cb < cend; cb += TRI_NW * KS) {
    double4_t x[KS];
    double a[KS][4];
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int c = cb + u * TRI_NW;
      const int k = 32 * c + 16 * h + 4 * g;
      const bool ok = c < cend && k < n;  // k + 3 stays inside the pitch (n rounded up to 16)
      x[u] = (double4_t){0.0, 0.0, 0.0, 0.0};
      if (rok && ok) x[u] = *reinterpret_cast<const double4_t*>(trow + k);
      if constexpr (VEC) {
        double4_t av = (double4_t){0.0, 0.0, 0.0, 0.0};
        if (fok && ok) av = *reinterpret_cast<const double4_t*>(irow + k);
#pragma unroll
        for (int s = 0; s < 4; ++s) a[u][s] = k + s < n ? av[s] : 0.0;
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) a[u][s] = (fok && ok && k + s < n) ? irow[k + s] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < KS; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][s], x[u][s], acc, 0, 0, 0);
  }
  // result register j of lane (r, g) is operand row g + 4 j (field f0 + (g + 4j) % 8, range
  // (g + 4j) / 8 = j / 2) times operand column r (row i0 + r % 8, range r / 8): lanes of range h
  // keep registers 2h and 2h + 1, entry h * 64 + 8 f + i of the wave's partial
  red[w][h * 64 + 8 * g + rr] = acc[2 * h];
  red[w][h * 64 + 8 * (g + 4) + rr] = acc[2 * h + 1];
  __syncthreads();
  if (tid < 64) {
    double s = 0.0;
#pragma unroll
    for (int v = 0; v < TRI_NW; ++v) s += red[v][tid] + red[v][64 + tid];
    const int f = f0 + (tid >> 3), i = i0 + (tid & 7);
    if (f < B && i < n) out[(int64_t)f * out_fs + i] = s;
  }
}

// the tile form of a product of n rows and B fields: 8 x 8 for up to 8 fields (a 16-field tile
// would stream twice the rows for the same fields) or few 16 x 16 tiles; 64 x 64 blocks for many
// fields and many tiles; else 16 x 16
int tri_form(int n, int B) {
  const int64_t tiles16 = (int64_t)((n + 15) / 16) * ((B + 15) / 16);
  if (B <= 8 || tiles16 <= TRI_FORM8_MAX_TILES) return TRI_FORM8;
  const int64_t blocks = (int64_t)((n + 63) / 64) * ((B + 63) / 64);
  if (B >= TRI_BLOCK_MIN_FIELDS && blocks >= TRI_BLOCK_MIN_TILES) return TRI_FORM_BLOCK;
  return TRI_FORM16;
}

// tile b of a launch in dispatch order -> (row tile, field group): heaviest row tiles first,
// field groups of one row tile next to each other
__device__ __forceinline__ void tri_tile_of(int b, int upper, int nt, int nfz, int* t, int* z) {
  const int tr = b / nfz;
  *z = b - tr * nfz;
  *t = upper ? tr : nt - 1 - tr;
}

template <int UPPER, bool VEC>
__global__ void __launch_bounds__(64 * TRI_NW) k_tri_tile(const double* __restrict__ T, int64_t ldt, int n,
                                                         const double* __restrict__ in, int64_t in_fs, int B,
                                                         double* __restrict__ out, int64_t out_fs) {
  __shared__ double red[TRI_NW][256];
  tri_tile_body<UPPER, VEC, 6>(T, ldt, n, in, in_fs, B, out, out_fs, blockIdx.x, blockIdx.y, red);
}

template <int UPPER, bool VEC>
__global__ void __launch_bounds__(64 * TRI_NW) k_tri_tile8(const double* __restrict__ T, int64_t ldt, int n,
                                                          const double* __restrict__ in, int64_t in_fs, int B,
                                                          double* __restrict__ out, int64_t out_fs, int nt, int nfz) {
  __shared__ double red[TRI_NW][256];
  int t, z;
  tri_tile_of(blockIdx.x, UPPER, nt, nfz, &t, &z);
  tri_tile8_body<UPPER, VEC, 4>(T, ldt, n, in, in_fs, B, out, out_fs, t, z, red);
}

// A workgroup barrier for LDS data only: this wave's LDS accesses complete, then the barrier.
// __syncthreads also waits for every outstanding global load (its workgroup fence), which would
// drain the chunks a pipelined loop keeps in flight.  The memory clobber keeps the compiler from
// moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Many fields and many tiles (the bandwidth regime): 64-row x 64-field block tiles, K staged
// through LDS 16 columns at a time, four waves each owning a 32 x 32 quadrant (2 x 2 MFMA tiles),
// as in the GEMM above.  A 16 x 16 tile reads (16 + 16) K doubles per 256 outputs; this one
// (64 + 64) K per 4096, a quarter of the cache traffic.  A block's chunks are a serial chain, so
// they go in groups of G = TRI_BLOCK_DEPTH: a group is stored to LDS, the next group's loads are
// issued, and the group's MFMAs run while they are in flight (one chunk ahead left every step
// waiting a memory latency).  Each tile's K range is its part of the
// triangle (rounded out to whole chunks; T is zero outside the triangle), the heaviest tiles
// first.
template <int UPPER>
__global__ void __launch_bounds__(256) k_tri_block(const double* __restrict__ T, int64_t ldt, int n,
                                                   const double* __restrict__ in, int64_t in_fs, int B,
                                                   double* __restrict__ out, int64_t out_fs, int ntn, int nfm) {
  constexpr int G = TRI_BLOCK_DEPTH;
  __shared__ double Is[G][16][64 + 1];  // [chunk of the group][k][field]
  __shared__ double Ts[G][16][64 + 1];  // [chunk of the group][k][row]
  const int tr = blockIdx.x / nfm, tm = blockIdx.x - tr * nfm;
  const int tn = UPPER ? tr : ntn - 1 - tr;
  const int f0 = 64 * tm, i0 = 64 * tn;
  const int kbeg = UPPER ? i0 : 0, kend = UPPER ? n : min(n, i0 + 64);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  double4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};
  // element e = tid + 256 q of a 64 x 16 chunk: row (field or T row) e / 16, column e % 16, so
  // 16 lanes read one 128-byte row segment
  const int ek = tid & 15, er = tid >> 4;
  double ra[G][4], rb[G][4];  // slot u holds chunk c0 + u of the next group
  // The loop has no branches and no value selects: the chunks run in whole groups of G and every
  // load is issued, from a clamped address.  Rows past n and fields past B read row n - 1 or
  // field B - 1: they only reach outputs that are not stored.  A column past the tile's range
  // (the triangle's edge, n, or chunks past the end) meets a zero of T: the strict triangle, or
  // the pitch padding (ldt > n, columns clamped to ldt - 1); its input value is any finite one
  // (column clamped to n - 1).  Conditional loads, or zeroing loaded values, made the compiler
  // wait for every outstanding load before each LDS store.
  auto fetch = [&](int c, double (&a)[4], double (&b)[4]) {
    const int k = kbeg + 16 * c + ek;
    const int kt = k < ldt ? k : (int)ldt - 1, ki = k < n ? k : n - 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = f0 + er + 16 * q, i = i0 + er + 16 * q;
      a[q] = in[(int64_t)(f < B ? f : B - 1) * in_fs + ki];
      b[q] = T[(int64_t)(i < n ? i : n - 1) * ldt + kt];
    }
  };
  const int nch = (kend - kbeg + 15) / 16;
#pragma unroll
  for (int u = 0; u < G; ++u) fetch(u, ra[u], rb[u]);
  for (int c0 = 0; c0 < nch; c0 += G) {
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        Is[u][ek][er + 16 * q] = ra[u][q];
        Ts[u][ek][er + 16 * q] = rb[u][q];
      }
    lds_barrier();  // the group is visible
#pragma unroll
    for (int u = 0; u < G; ++u) fetch(c0 + G + u, ra[u], rb[u]);
    // the operands of step t + 1 are read from LDS before step t's MFMAs issue, so the reads'
    // latency overlaps the MFMA pipe instead of draining it
    {
      const int kq0 = lane >> 4, m = lane & 15;
      double op[2][4];
      op[0][0] = Is[0][kq0][wm + m];
      op[0][1] = Is[0][kq0][wm + 16 + m];
      op[0][2] = Ts[0][kq0][wn + m];
      op[0][3] = Ts[0][kq0][wn + 16 + m];
#pragma unroll
      for (int t = 0; t < 4 * G; ++t) {
        const int cur = t & 1, nxt = cur ^ 1;
        if (t + 1 < 4 * G) {
          const int u = (t + 1) >> 2, kq = 4 * ((t + 1) & 3) + kq0;
          op[nxt][0] = Is[u][kq][wm + m];
          op[nxt][1] = Is[u][kq][wm + 16 + m];
          op[nxt][2] = Ts[u][kq][wn + m];
          op[nxt][3] = Ts[u][kq][wn + 16 + m];
        }
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[cur][0], op[cur][2], acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[cur][0], op[cur][3], acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[cur][1], op[cur][2], acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[cur][1], op[cur][3], acc[1][1], 0, 0, 0);
      }
    }
    lds_barrier();  // every wave is done with the group before the next one is stored
  }
  // result register r of lane l in quadrant tile (i, j): field f0 + wm + 16 i + l / 16 + 4 r,
  // row i0 + wn + 16 j + l % 16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = f0 + wm + 16 * i + (lane >> 4) + 4 * r, row = i0 + wn + 16 * j + (lane & 15);
        if (f < B && row < n) out[(int64_t)f * out_fs + row] = acc[i][j][r];
      }
}

// Persistent form for an uneven batch: the tiles of several problems' products in one list
// (problem i owns tiles [first[i], first[i + 1])), walked by a grid of about one resident
// round of workgroups, workgroup b taking tiles b, b + grid, ...  Tile (t, z) of a problem
// computes what the problem's own launch computes.
template <typename T> using const_as = const __attribute__((address_space(4))) T;

template <int UPPER, bool VEC, bool F8>
__global__ void __launch_bounds__(64 * TRI_NW) k_tri_tile_queue(TriQueue qa) {
  __shared__ double red[TRI_NW][256];
  int prob = 0, iter = 0;
  for (;;) {
    // the tile index only grows, so the problem is found by stepping forward from the last one
    const int tile = blockIdx.x + (iter++) * gridDim.x;
    if (tile >= qa.total) return;
    while (prob + 1 < qa.count && qa.first[prob + 1] <= tile) ++prob;
    const_as<TriProb>* p = (const_as<TriProb>*)(qa.probs) + prob;
    const int local = tile - qa.first[prob];
    if constexpr (F8) {
      int t, z;
      tri_tile_of(local, UPPER, p->nt, p->nfz, &t, &z);
      tri_tile8_body<UPPER, VEC, 4>(p->T, p->ldt, p->n, p->in, p->in_fs, p->B, p->out, p->out_fs, t, z, red);
    } else {
      tri_tile_body<UPPER, VEC, 5>(p->T, p->ldt, p->n, p->in, p->in_fs, p->B, p->out, p->out_fs, local % p->nt,
                                local / p->nt, red);
    }
    __syncthreads();  // red is reused by the next tile
  }
}

TriProb tri_prob(const double* T, int64_t ldt, int n, const double* in, int64_t in_fs, double* out, int64_t out_fs,
                 int B) {
  TriProb p{};
  p.T = T;
  p.ldt = ldt;
  p.in = in;
  p.in_fs = in_fs;
  p.out = out;
  p.out_fs = out_fs;
  p.n = n;
  p.B = B;
  p.form = tri_form(n, B);
  if (p.form == TRI_FORM_BLOCK && ldt <= n) p.form = TRI_FORM16;  // the block form needs a zero pad column
  const int rows = p.form == TRI_FORM8 ? 8 : p.form == TRI_FORM_BLOCK ? 64 : 16;
  p.nt = (n + rows - 1) / rows;
  p.nfz = (B + rows - 1) / rows;
  p.vec = (in_fs & 3) == 0 && (reinterpret_cast<uintptr_t>(in) & 31) == 0;
  return p;
}

static int cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess || cus < 1)
    cus = 1;
  return cus;
}

template <typename K>
static int tri_resident(K kernel) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 64 * TRI_NW, 0) != hipSuccess || per < 1) per = 1;
  return per * cu_count();
}

hipError_t tri_apply_queue(const TriQueue& q, int upper, int vec, int form, hipStream_t st) {
  const int form8 = form == TRI_FORM8;
  if (form != TRI_FORM8 && form != TRI_FORM16) return hipErrorInvalidValue;
#define KRIG_TRIQ(U, V, F)                                                                                  \
  if (upper == U && vec == V && form8 == F) {                                                               \
    hipLaunchKernelGGL((k_tri_tile_queue<U, V, F>), dim3(tri_resident(k_tri_tile_queue<U, V, F>)),            \
                       dim3(64 * TRI_NW), 0, st, q);                                                        \
    return hipGetLastError();                                                                               \
  }
  KRIG_TRIQ(0, true, 0) KRIG_TRIQ(0, false, 0) KRIG_TRIQ(1, true, 0) KRIG_TRIQ(1, false, 0)
  KRIG_TRIQ(0, true, 1) KRIG_TRIQ(0, false, 1) KRIG_TRIQ(1, true, 1) KRIG_TRIQ(1, false, 1)
#undef KRIG_TRIQ
  return hipErrorInvalidValue;
}

hipError_t tri_apply(const double* T, int64_t ldt, int n, int upper, const double* in, int64_t in_fs, double* out,
                     int64_t out_fs, int B, hipStream_t st) {
  if (n <= 0 || B <= 0) return hipSuccess;
  if ((ldt & 3) || ldt < (int64_t)(n + 15) / 16 * 16 || (reinterpret_cast<uintptr_t>(T) & 31))
    return hipErrorInvalidValue;
  return tri_apply_prob(tri_prob(T, ldt, n, in, in_fs, out, out_fs, B), upper, st);
}

hipError_t tri_apply_prob(const TriProb& p, int upper, hipStream_t st) {
  if (p.form == TRI_FORM_BLOCK) {
    if (upper)
      hipLaunchKernelGGL(k_tri_block<1>, dim3(p.nt * p.nfz), dim3(256), 0, st, p.T, p.ldt, p.n, p.in, p.in_fs, p.B,
                         p.out, p.out_fs, p.nt, p.nfz);
    else
      hipLaunchKernelGGL(k_tri_block<0>, dim3(p.nt * p.nfz), dim3(256), 0, st, p.T, p.ldt, p.n, p.in, p.in_fs, p.B,
                         p.out, p.out_fs, p.nt, p.nfz);
    return hipGetLastError();
  }
#define KRIG_TRI(U, V)                                                                                        \
  if (upper == U && p.vec == V) {                                                                             \
    if (p.form == TRI_FORM8)                                                                                  \
      hipLaunchKernelGGL((k_tri_tile8<U, V>), dim3(p.nt * p.nfz), dim3(64 * TRI_NW), 0, st, p.T, p.ldt, p.n,   \
                         p.in, p.in_fs, p.B, p.out, p.out_fs, p.nt, p.nfz);                                    \
    else                                                                                                      \
      hipLaunchKernelGGL((k_tri_tile<U, V>), dim3(p.nt, p.nfz), dim3(64 * TRI_NW), 0, st, p.T, p.ldt, p.n,     \
                         p.in, p.in_fs, p.B, p.out, p.out_fs);                                                 \
    return hipGetLastError();                                                                                 \
  }
  KRIG_TRI(0, true) KRIG_TRI(0, false) KRIG_TRI(1, true) KRIG_TRI(1, false)
#undef KRIG_TRI
  return hipErrorInvalidValue;
}

}  // namespace krig
