// Argument blocks and the per-size kernel table of the two-level FFT passes.
//
// A transform of length F = N1 * N2 is done in two register stages joined by one
// LDS exchange (Cooley-Tukey "four-step" split): with n = N2*n1 + n2 and
// k = k1 + N1*k2,
//   X[k1 + N1 k2] = sum_n2 W_N2^(n2 k2) W_F^(n2 k1) sum_n1 x[N2 n1 + n2] W_N1^(n1 k1).
// Stage A: one thread per n2 holds x[N2 n1 + n2] for all n1, does the length-N1
// DFT and the twiddle W_F^(n2 k1); stage B: one thread per k1 holds all n2 and
// does the length-N2 DFT, ending with X[k1 + N1 k2] for all k2 in registers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace krig {

// Two-window selection of rows or columns: indices [a0, a0+na) go to destination
// 0.., and [b0, b0+nb) to destination na.. (nb may be 0).
struct Window {
  int a0, na, b0, nb;
};

// Forward real-row transform (two rows per complex line), output half spectrum.
struct RowsR2CArgs {
  int nrows;             // rows of the (virtual) input image
  int H2, ldH;           // half-spectrum length F/2+1 and output row pitch
  void* out;             // cx<TS> [B][nrows][ldH]
  int64_t out_fs;        // field stride of out (elements)
  const void* twF;       // cx<TC> [F] forward twiddles exp(-2 pi i j/F)
  // source CSR (scatter of alpha_i * w_im onto the padded grid)
  const int32_t* row_ptr;   // [nrows*ncols + 1]
  const int32_t* ent_site;  // [nnz]
  const double* ent_w;      // [nnz]
  const double* alpha;      // [B][n]
  int64_t alpha_fs;
  // dense source: in[b][r][c] placed at column offset coff (valid cols ncols)
  const void* dense;        // TS
  int64_t dense_fs, dense_ld;
  int coff;
  int ncols;                // nonzero columns of the input rows
  // even-reflected lag source: row r of the F1 x F2 embedding of lag[n1l][n2l]
  const double* lag;
  int n1l, n2l, F1;
  int NL;                   // lines (row pairs) per block
};

// Column pass: forward FFT, optional multiply by the real filter, inverse FFT.
struct ColsArgs {
  int H2;                 // number of columns
  int ldH;                // pitch of the column-major-by-rows arrays (row pitch)
  const void* in;         // cx<TS> [B][*][ldH]
  int64_t in_fs;
  int in_off, in_cnt;     // input row r sits at FFT index r + in_off
  const void* in2;        // second input (dlag: c* spectrum rows) cx<TS>
  int64_t in2_fs;
  int in2_off, in2_cnt;
  const void* filt;       // TS [F][ldH] real filter (already scaled by 1/(F1 F2))
  void* out;              // cx<TS> [B][*][ldH]
  int64_t out_fs;
  Window rows;            // FFT-index rows to keep
  void* part;             // cx<TS> [ngroups][F][ldH] dlag partial spectra
  int G;                  // fields per block (dlag)
  int B;                  // total fields
  const void* twF;        // cx<TF> [F] twiddles of the forward transform's precision
  const void* twI;        // cx<TI> [F] twiddles of the inverse transform's precision
  double scale;           // store scale (setup transforms)
  int NL;                 // columns per block
};

// Inverse real-row transform (two rows per complex line) from a half spectrum.
struct RowsC2RArgs {
  int nrows;
  int H2, ldH;
  const void* in;         // cx<TS> [B][nrows][ldH]
  int64_t in_fs;
  void* out;              // TS [B][nrows][ldo]
  int64_t out_fs, ldo;
  Window cols;            // FFT-index columns to keep
  const void* add;        // optional TS image added to the output: add[b][r + add_r0][c + add_c0]
  int64_t add_fs, add_ld;
  int add_r0, add_c0;
  const void* twF;        // cx<TC> [F]
  int NL;
};

typedef hipError_t (*launch_rows_r2c_t)(const RowsR2CArgs&, int B, hipStream_t);
typedef hipError_t (*launch_cols_t)(const ColsArgs&, int nblk_y, hipStream_t);
typedef hipError_t (*launch_rows_c2r_t)(const RowsC2RArgs&, int B, hipStream_t);

// Kernels for one transform length.  Arithmetic and storage precisions are fixed
// per role: everything is FP64 except the inverse half of the prediction's column
// pass and the prediction's inverse rows in the FP32 form.
struct FftSet {
  launch_rows_r2c_t r2c_csr;        // scatter + forward rows, FP64 -> FP64 spectra
  launch_rows_r2c_t r2c_dense_f32;  // FP32 rows (upstream gradient) -> FP64 spectra
  launch_rows_r2c_t r2c_dense_f64;  // FP64 rows -> FP64 spectra
  launch_rows_r2c_t r2c_lag;        // even-reflected lag quadrant, FP64
  launch_cols_t conv_mixed;         // FP64 forward, x filter, FP32 inverse, FP32 out
  launch_cols_t conv64;             // all FP64
  launch_cols_t conv_dlag64;        // all FP64, plus sum_b G_b conj(C_b) partial spectra
  launch_cols_t fwd_real64;         // forward columns, store Re * scale (FP64)
  launch_cols_t inv_sum64;          // inverse columns of a sum of partial spectra (FP64)
  launch_rows_c2r_t c2r32;          // inverse rows, FP32
  launch_rows_c2r_t c2r64;          // inverse rows, FP64
};

struct FftEntry {
  int F, N1, N2;
  FftSet k;
};

// size registry (filled by the generated per-size translation units)
void register_fft(const FftEntry& e);
const FftEntry* find_fft(int F);
int fft_sizes(int* out, int cap);
void register_all_fft();

}  // namespace krig
