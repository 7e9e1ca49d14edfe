// Set-up and gather/scatter kernels of the rapid predictor (Section 2.2, Steps 1-6).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "matern_dev.h"

namespace krig {

struct GridDev {
  int m1, m2, L;
  double x0, y0, dx, dy;
  int P1, P2, M;
};

// lag[a][b] = k((a dx, b dy)), a < m1+L, b < m2+L (Step 2's filter on its quadrant)
hipError_t lag_image(const GridDev& g, const MaternDev& mt, double* lag64, hipStream_t st);
// FP64 -> storage precision copies
hipError_t convert_f64(const double* src, void* dst, int64_t cnt, int to_f32, hipStream_t st);
hipError_t convert_to_f64(const void* src, double* dst, int64_t cnt, int from_f32, hipStream_t st);
// 2D copy with pitch: dst[r][c] = src[r][c] (r < nr, c < nc) as storage type
hipError_t copy2d_f64_to(const double* src, int64_t lds_, void* dst, int64_t ldd, int nr, int nc, int to_f32,
                         hipStream_t st);

// Step 1: K_N (M x M) from the neighbour offsets, its Cholesky factor and the inverse
// factor LinvN = L_N^{-1}.  One block.  On a non-positive pivot the factorisation is
// retried once with jitter 1e-14*sigma2*M on the diagonal; status bit 1 = jitter used,
// status = -(pivot+1) if the retry fails too.
hipError_t kn_factor(const GridDev& g, const MaternDev& mt, double* KN, double* LinvN, int* status,
                     hipStream_t st);
// K_N for more than 64 neighbours (L > 4), for the blocked factorisation: KN (may be NULL)
// receives K_N, A receives K_N + jit I (both M x M row-major).
hipError_t kn_assemble(const GridDev& g, const MaternDev& mt, double* KN, double* A, double jit, hipStream_t st);
// Step 3: anchor cell (i0, j0) and k_i (n x M) of every site; sites [n][2] FP64.
hipError_t site_kvec(const GridDev& g, const MaternDev& mt, const double* sites, int n, int32_t* anchor,
                     double* kvec, hipStream_t st);
// W [n][M] -> Wt [M][n] in gather order: Wt[m][s] = W[order[s]][m] (order NULL: the identity).
// The gathers walk sites in that order (slot s holds site order[s]): with the sites sorted by
// anchor cell, neighbouring lanes read neighbouring image windows and share cache lines.
hipError_t transpose_w(const double* W, int n, int M, const int32_t* order, double* Wt, hipStream_t st);

// Step 5 structure: CSR over the padded grid (deterministic, no float atomics).
//  cell_cnt [m1*m2], cell_ptr [m1*m2+1], cell_sites [n], node_ptr [P1*P2+1],
//  ent_site [n*M], ent_w [n*M]; scan_tmp: >= 2*(P1*P2/256+2) ints.
struct CsrWork {
  int32_t *cell_cnt, *cell_ptr, *cell_cur, *cell_sites, *node_cnt, *scan_tmp;
};
hipError_t build_csr(const GridDev& g, const int32_t* anchor, const double* W, int n, const CsrWork& w,
                     int32_t* node_ptr, int32_t* ent_site, double* ent_w, hipStream_t st);
// Rewrite the entry weights of an existing scatter structure from new weights W [n][M]
// whose anchors are unchanged (the node pointers and entry sites stay as they are):
// ent_w[e] = W[site][m] with m the offset of the entry's node from the site's anchor.
hipError_t refill_csr_weights(const GridDev& g, const int32_t* anchor, const double* W,
                              const int32_t* node_ptr, const int32_t* ent_site, double* ent_w, hipStream_t st);

// c* image [B][P1][P2] (storage precision) = A^T alpha by segment sums (FP64 accumulation)
hipError_t scatter_image(const GridDev& g, const int32_t* node_ptr, const int32_t* ent_site, const double* ent_w,
                         const double* alpha, int64_t alpha_fs, int B, void* img, int64_t img_fs, int to_f32,
                         hipStream_t st);
// out[b][i] = sum_m W[i][m] img[b][(i0+L+ox_m) * ldi + j0+L+oy_m] (FP64 accumulation, in the
// order of m), with Wt the transposed weights in the gather order `order` (transpose_w; NULL:
// the identity); the sites are visited in that order, each writing its own output.  `anchor`
// holds the anchors (i0, j0) in the same order: slot s reads anchor[2s], anchor[2s + 1] and
// writes site order[s].
// csim_residual: out[r][i] = y[i] - (that + noise_sd * N(0,1) Philox noise of (i, r0 + r)).
hipError_t gather_sites(const GridDev& g, const int32_t* anchor, const double* Wt, const int32_t* order, int n,
                        const void* img, int64_t img_fs, int64_t ldi, int B, int from_f32, double* out,
                        int64_t out_fs, hipStream_t st);
hipError_t csim_residual(const GridDev& g, const int32_t* anchor, const double* Wt, const int32_t* order, int n,
                         const void* img, int64_t img_fs, int64_t ldi, int R, int from_f32, const double* y,
                         double noise_sd, uint64_t seed, int r0, double* out, int64_t out_fs, hipStream_t st);

// circulant-embedding eigenvalues: per-block min / max / negative count (the host
// finishes the reduction), then x <- sqrt(max(x, 0) * scale)
hipError_t minmax_blocks(const double* x, int64_t cnt, double* bmin, double* bmax, int* bneg, int nblocks,
                         hipStream_t st);
hipError_t sqrt_clamp(double* x, int64_t cnt, double scale, hipStream_t st);
// x <- x / d (the reflection-free filter set-up divides out the centre's phase)
hipError_t div_f64(double* x, const double* d, int64_t cnt, hipStream_t st);

}  // namespace krig
