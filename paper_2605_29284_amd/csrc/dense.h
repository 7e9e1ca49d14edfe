// FP64 dense linear algebra kernels (GPU) used for the kriging system.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "matern_dev.h"

namespace krig {

struct GemmArgs {
  const double* A;
  int64_t lda;
  int transA;
  const double* B;
  int64_t ldb;
  int transB;
  double* C;
  int64_t ldc;
  int m_off, M_end;   // rows [m_off, M_end) of C (and of op(A))
  int n_off, N_end;   // cols [n_off, N_end) of C (and of op(B))
  int K;
  double alpha, beta;
  int lower;          // only tiles with tile_col <= tile_row, and entries col <= row
};

hipError_t gemm_f64(const GemmArgs& g, hipStream_t st);
hipError_t assemble_kt(const double* d_sites, int n, const MaternDev& mt, double* Kt, int64_t ld,
                       hipStream_t st);
hipError_t cholesky_and_inverse(double* A, int64_t lda, int n, double* Linv, double* Dinv, double* work,
                                int* d_status, hipStream_t st);
hipError_t copy_rows(const double* src, int64_t ld_src, double* dst, int64_t ld_dst, int nr, int nc,
                     hipStream_t st);
hipError_t fill_f64(double* p, int64_t cnt, double v, hipStream_t st);
// dst = src^T for an n x n matrix
hipError_t transpose_f64(const double* src, int64_t ld_src, double* dst, int64_t ld_dst, int n, hipStream_t st);
// out[b] = T in[b] for a triangular T (upper = 0: lower, 1: upper); T row-major with a
// pitch ldt that is a multiple of 4 and >= n rounded up to 16, 32-byte aligned, zeros
// outside the triangle and in the padding.  hipErrorInvalidValue otherwise.  One launch,
// no workspace; in and out must not overlap.
hipError_t tri_apply(const double* T, int64_t ldt, int n, int upper, const double* in, int64_t in_fs, double* out,
                     int64_t out_fs, int B, hipStream_t st);

// Tile forms of the triangular products (tri_form): 16-row x 16-field tiles; 8 x 8 tiles for
// products of up to 8 fields or with at most TRI_FORM8_MAX_TILES 16 x 16 tiles; 64 x 64 block
// tiles for products of TRI_BLOCK_MIN_FIELDS fields or more with at least TRI_BLOCK_MIN_TILES
// of them (a block's chunks are a serial chain: fewer blocks leave compute units idle) when T has
// a zero pad column (ldt > n).  A product's bits depend on its form.
enum { TRI_FORM16 = 0, TRI_FORM8 = 1, TRI_FORM_BLOCK = 2 };
constexpr int TRI_FORM8_MAX_TILES = 128;
constexpr int TRI_BLOCK_MIN_FIELDS = 64;
constexpr int TRI_BLOCK_MIN_TILES = 256;
constexpr int TRI_BLOCK_DEPTH = 4;  // chunks in flight per block
int tri_form(int n, int B);

// One problem of a persistent triangular product (an uneven batch): tri_apply's arguments and
// its tile counts (nt row tiles x nfz field groups of the tile form; vec: 32-byte input vectors).
struct TriProb {
  const double* T;
  int64_t ldt;
  const double* in;
  int64_t in_fs;
  double* out;
  int64_t out_fs;
  int n, B, nt, nfz, vec, form;
};
TriProb tri_prob(const double* T, int64_t ldt, int n, const double* in, int64_t in_fs, double* out, int64_t out_fs,
                 int B);
struct TriQueue {
  const TriProb* probs;   // device array of count problems
  const int* first;       // [count + 1] prefix sums of their tile counts (nt nfz each)
  int count, total;
};
// one problem's product in its own launch (what tri_apply launches)
hipError_t tri_apply_prob(const TriProb& p, int upper, hipStream_t st);
// the products of problems that all have this (upper, vec, form), form TRI_FORM16 or TRI_FORM8
hipError_t tri_apply_queue(const TriQueue& q, int upper, int vec, int form, hipStream_t st);

}  // namespace krig
