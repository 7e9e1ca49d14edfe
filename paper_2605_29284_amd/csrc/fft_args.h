// Argument blocks, geometry and the per-size kernel table of the FFT passes.
//
// A transform of length F = R1 * R2 * R3 runs in up to three register stages joined
// by LDS exchanges.  With M = R2 * R3, n = m + M j and k = k1 + R1 k',
//   X[k1 + R1 k'] = sum_m W_M^(m k') W_F^(m k1) sum_j x[m + M j] W_R1^(j k1)
// (pass 1: one thread per m does the length-R1 DFT over j and the twiddle), and each
// of the R1 inner length-M transforms is split again as M = R2 * R3 (Cooley-Tukey
// "four-step"): with m = R3 n1 + s and k' = s' + R2 k2,
//   Z[s' + R2 k2] = sum_s W_R3^(s k2) W_M^(s s') sum_n1 z[R3 n1 + s] W_R2^(n1 s').
// R1 = 1 is the two-stage form.  Between passes the data cross lanes through LDS.
//
// Register layouts:  input  thread t < TIN  holds x[t + TIN j],  j < NIN;
//                    output thread t < TOUT holds X[t + TOUT k], k < NOUT = R3.
// The inverse transform can start from the output layout and end in the input
// layout, so a forward/inverse pair needs no reordering in between.
//
// Half spectra between the row and column passes are stored frequency-major:
// element (field b, frequency k, row r) at base + b*fs + k*ld + r, so that a
// column pass reads and writes whole contiguous columns.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace krig {

// Two-window selection of rows or columns: indices [a0, a0+na) go to destination
// 0.., and [b0, b0+nb) to destination na.. (nb may be 0).
struct Window {
  int a0, na, b0, nb;
};

// Forward real-row transform (two rows per complex line); output: half spectra,
// frequency-major.
struct RowsR2CArgs {
  int nrows;             // rows of the (virtual) input image
  int H2;                // half-spectrum length F/2+1
  void* out;             // cx<TS>: out[b*out_fs + k*out_ld + r]
  int64_t out_fs, out_ld;
  const void* twF;       // cx<TC> [F] forward twiddles exp(-2 pi i j/F)
  // source CSR (scatter of alpha_i * w_im onto the padded grid)
  const int32_t* row_ptr;   // [nrows*ncols + 1]
  const int32_t* ent_site;  // [nnz]
  const double* ent_w;      // [nnz]
  const double* alpha;      // [B][n]
  int64_t alpha_fs;
  const double* alpha_scale;  // [n] per-site factor of alpha (the scaled scatter only)
  // dense source: in[b][r][c] (row-major) placed at column offset coff
  const void* dense;        // TIN
  int64_t dense_fs, dense_ld;
  int coff;
  int ncols;                // nonzero columns of the input rows
  // even-reflected lag source: row r of the F1 x F2 embedding of lag[n1l][n2l]
  const double* lag;
  int n1l, n2l, F1;
  // covariance on the F1 x F2 torus (minimal-image lags) for circulant embedding
  double cov_sigma2, cov_rho, cov_dx, cov_dy;
  int cov_kind;
  int NL;                   // lines (row pairs) per block
};

// Column pass over frequency-major half spectra: forward transform, optional
// product with the real filter spectrum, inverse transform.
struct ColsArgs {
  int H2;                 // number of columns (frequencies)
  const void* in;         // cx<TSI>: in[b*in_fs + c*in_ld + r]
  int64_t in_fs, in_ld;
  int in_off, in_cnt;     // input row r sits at transform index r + in_off
  const void* in2;        // second input (lag gradient: row spectra of c*)
  int64_t in2_fs, in2_ld;
  int in2_off, in2_cnt;
  const void* filt;       // TF filt[c*filt_ld + k], already scaled by 1/(F1 F2)
  int64_t filt_ld;
  void* out;              // cx<TSO>: out[b*out_fs + c*out_ld + d]
  int64_t out_fs, out_ld;
  Window rows;            // transform-index rows to keep
  void* part;             // cx<TSO> part[g*part_fs + c*part_ld + k] (lag-gradient partial spectra)
  int64_t part_fs, part_ld;
  int G;                  // number of partials (inverse sum)
  int B;                  // total fields
  const void* twF;        // cx<TF> [F] twiddles of the forward transform's precision
  const void* twI;        // cx<TI> [F] twiddles of the inverse transform's precision
  double scale;           // store scale (set-up transforms)
  // circulant-embedding sampler: complex Philox noise x sqrt(Lambda / N) on the torus
  uint32_t key0, key1;    // Philox key (seed)
  int pair0;              // first realisation pair of this launch
  int ncol_full;          // torus length along the columns' index (all frequencies)
  int NL;                 // columns per block
};

// Circulant-embedding sampler, second pass: complex transforms of torus rows
// (frequency-major input) -> realisations 2p (real part) and 2p+1 (imaginary part).
struct RowsCEArgs {
  int nrows;              // rows kept (P1)
  int ncols;              // torus row length (all frequencies)
  const void* in;         // cx<TS>: in[pair*in_fs + k*in_ld + r]
  int64_t in_fs, in_ld;
  void* out;              // TO [R][nrows][ldo]
  int64_t out_fs, ldo;
  int keep;               // columns kept (P2)
  int R, pair0;
  const void* twF;
  int NL;
};

// Inverse real-row transform (two rows per complex line) from frequency-major half
// spectra; output rows are row-major.
struct RowsC2RArgs {
  int nrows;
  int H2;
  const void* in;         // cx<TS>: in[b*in_fs + k*in_ld + r]
  int64_t in_fs, in_ld;
  void* out;              // TO [B][nrows][ldo]
  int64_t out_fs, ldo;
  Window cols;            // transform-index columns to keep
  const void* add;        // optional TO image added to the output: add[b][r + add_r0][c + add_c0]
  int64_t add_fs, add_ld;
  int add_r0, add_c0;
  const void* twF;        // cx<TC> [F]
  double scale;           // output scale (folded form)
  int NL;
};

// Inverse rows of a spatially weighted mixture: out[b][r][c] = sum_{k < C} lam[k][r][c] *
// (inverse rows of component k's spectra)[b][r][c], accumulated in FP64 in component order
// and rounded once.  The components share the geometry of r (their spectra differ only in
// their base pointer); r.in and r.add are not used.
constexpr int MIX_COMP_MAX = 8;
struct MixRowsArgs {
  RowsC2RArgs r;
  const void* in[MIX_COMP_MAX];   // component k's spectra, laid out as r.in_fs / r.in_ld
  const double* lam;              // lam[k * lam_cs + r * lam_ld + c]
  int64_t lam_cs, lam_ld;
  int C;
};

// Persistent launch over several problems of one transform form (an uneven batch): problem
// i's argument block is args[i] (RowsR2CArgs, ColsArgs or RowsC2RArgs, all with the same NL),
// its tiles are [first[i], first[i + 1]) of the list, nbx[i] per field.
struct QueueArgs {
  const void* args;       // device array of count argument blocks
  const int* first;       // [count + 1] prefix sums of the problems' tile counts
  const int* nbx;         // [count] row or column blocks per field
  int count, total;
};

typedef hipError_t (*launch_rows_r2c_t)(const RowsR2CArgs&, int B, hipStream_t);
typedef hipError_t (*launch_cols_t)(const ColsArgs&, int nblk_y, hipStream_t);
typedef hipError_t (*launch_rows_c2r_t)(const RowsC2RArgs&, int B, hipStream_t);
typedef hipError_t (*launch_rows_c2r_mix_t)(const MixRowsArgs&, int B, hipStream_t);
typedef hipError_t (*launch_rows_ce_t)(const RowsCEArgs&, int npairs, hipStream_t);
// nblocks 0: one resident round of blocks (occupancy x compute units), -d: a d-th of it
typedef hipError_t (*launch_queue_t)(const QueueArgs&, int NL, int nblocks, hipStream_t);

// Kernels for one transform length.  Arithmetic is FP64 in every role of the
// prediction and its adjoint.  FP64 plans store FP64 spectra between the passes; FP32
// plans store the column pass's output of the prediction in FP32 and every other spectrum
// in FP64 (spec_bytes in plan.cpp gives the reasons).
// Only the conditional-simulation sampler has an FP32-arithmetic form.
struct FftSet {
  launch_rows_r2c_t r2c_csr;        // scatter + forward rows, FP64 -> FP64 spectra
  launch_rows_r2c_t r2c_csr_scaled; //   ... of alpha[b][i] * alpha_scale[i] (mixture components)
  launch_rows_r2c_t r2c_dense_f32;  // FP32 rows (upstream gradient) -> FP64 spectra
  launch_rows_r2c_t r2c_dense_f64;  // FP64 rows -> FP64 spectra
  launch_rows_r2c_t r2c_lag;        // even-reflected lag quadrant, FP64
  launch_cols_t conv64;             // all FP64
  launch_cols_t conv_pred_f;        // FP32 plans' prediction: FP64 row spectra in, FP32 out
  launch_cols_t conv_dlag64;        // all FP64, plus sum_b G_b conj(C_b) partial spectra (NL fields
                                    // of one column per block, one partial per block row)
  launch_cols_t fwd_real64;         // forward columns, store Re * scale (FP64)
  launch_cols_t inv_sum64;          // inverse columns of a sum of partial spectra (FP64)
  launch_rows_c2r_t c2r64;          // inverse rows, FP64
  launch_rows_c2r_t c2r_f32;        // inverse rows, FP32 spectra -> FP32 output (FP64 arithmetic)
  launch_rows_c2r_mix_t c2r_mix64;  // weighted sum of components' inverse rows, FP64
  launch_rows_c2r_mix_t c2r_mix_f32;//   ... FP32 spectra and output (FP64 arithmetic)
  launch_rows_c2r_t c2r_fold32;     // inverse rows of the compact correlation, sign images
  launch_rows_c2r_t c2r_fold64;     //   folded, FP64 arithmetic -> FP32 / FP64 lag gradient
  launch_rows_r2c_t r2c_cov;        // covariance on the embedding torus, FP64
  launch_rows_r2c_t r2c_center;     // covariance about the torus centre (F1/2, F2/2), plain coordinates
  launch_rows_r2c_t r2c_delta;      // indicator of the torus centre
  // persistent forms of the prediction's passes (uneven batches)
  launch_queue_t q_r2c_csr, q_conv64, q_c2r64, q_conv_pred_f, q_c2r_f32;
  launch_queue_t q_r2c_dense;  // forward rows of FP64 images (problems whose scatter runs apart)
  launch_cols_t ce_cols32, ce_cols64;    // sampler pass 1 (noise x sqrt(Lambda), column transforms)
  launch_rows_ce_t ce_rows32, ce_rows64; // sampler pass 2 (row transforms -> two realisations)
  // paired columns of twice this length (one wave per column, no block barriers), FP64 or
  // FP32 output spectra; set only for three-pass lengths on exactly 64 threads
  launch_cols_t pair_conv64 = nullptr, pair_conv_pred_f = nullptr;
  launch_queue_t q_pair_conv64 = nullptr, q_pair_conv_pred_f = nullptr;
  int pair_ex = 0;  // LDS slots per column of the paired kernels
};

__host__ __device__ constexpr int odd_up(int x) { return x | 1; }
__host__ __device__ constexpr int imax(int a, int b) { return a > b ? a : b; }

struct FftGeo {
  int R1, R2, R3;
  int F, M;         // length and inner length R2 * R3
  int NIN, TIN;     // input layout
  int NOUT, TOUT;   // output layout
  int T2;           // threads of the middle pass (R1 * R3)
  int NT;           // threads per line
  int ON2;          // odd stride between the R3 rows of an inner exchange
  int RS;           // odd size of one inner exchange region
  int P1;           // row stride of the pass-1 exchange (at least M, = R3 mod 16)
  int EX;           // LDS slots per line for the exchanges
  int ROWS;         // row kernels: exchanges, natural-order pairing or transpose
};

__host__ __device__ constexpr FftGeo fft_geo(int R1, int R2, int R3) {
  FftGeo g{};
  g.R1 = R1;
  g.R2 = R2;
  g.R3 = R3;
  g.F = R1 * R2 * R3;
  g.M = R2 * R3;
  g.NIN = R1 > 1 ? R1 : R2;
  g.TIN = R1 > 1 ? g.M : R3;
  g.NOUT = R3;
  g.TOUT = R1 * R2;
  g.T2 = R1 * R3;
  g.NT = imax(imax(g.TIN, g.T2), g.TOUT);
  g.ON2 = odd_up(R2);
  g.RS = odd_up(R3 * g.ON2);
  // P1 = R3 (mod 16): the middle pass's lane t2 = (k1, s) = (t2 / R3, t2 mod R3) reads slot
  // k1 P1 + R3 n1 + s, which is t2 mod 16 plus a constant, so sixteen consecutive lanes use
  // sixteen different bank groups of 16 bytes (M + 1 put two rows one slot apart)
  g.P1 = g.M + ((g.R3 - g.M) % 16 + 16) % 16;
  g.EX = R1 > 1 ? imax(R1 * g.P1, R1 * g.RS) : g.RS;
  g.ROWS = imax(g.EX, g.F + 2);
  return g;
}

struct FftEntry {
  int F;
  FftGeo geo;
  FftSet k;
};

// size registry (filled by the generated per-size translation units)
void register_fft(const FftEntry& e);
const FftEntry* find_fft(int F);
// every compiled form of length F, the default first; returns the count
int fft_variants(int F, const FftEntry** out, int cap);
int fft_sizes(int* out, int cap);
void register_all_fft();

// LDS bytes of one block (lines or columns NL) for each kernel family
// Pitch of an LDS transpose with R values per k: R, padded by one where R is a multiple
// of 4 but not a power of two (the bank-group reasoning is at the transposes in
// fft_passes.h).
__host__ __device__ constexpr int tpitch(int R) { return (R % 4 == 0 && (R & (R - 1)) != 0) ? R + 1 : R; }
// Row kernels hold either NL lines or the block's transpose [k][2 NL] (k <= F/2); the
// circulant-embedding row kernel NL lines or a transpose [k][NL] (k < F).
inline size_t rows_lds(const FftGeo& g, int NL, size_t csz) {
  return (size_t)imax(NL * g.ROWS, (g.F / 2 + 1) * tpitch(2 * NL)) * csz;
}
inline size_t cols_lds(const FftGeo& g, int NL, size_t csz) { return (size_t)NL * g.EX * csz; }
inline size_t ce_rows_lds(const FftGeo& g, int NL, size_t csz) {
  return (size_t)imax(NL * imax(g.EX, g.F), g.F * tpitch(NL)) * csz;
}

}  // namespace krig
