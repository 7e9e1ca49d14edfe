// Two-level FFT pass kernels for the circulant-embedded convolution (Step 7) and
// its adjoint.  Included by one generated translation unit per transform length.
//
// Roles (TC/TF/TI = arithmetic precision, TS/TSI/TSO/TO = storage precision):
//  k_rows_r2c   forward transform of real rows, two rows per complex line
//               ("two-for-one"); sources: the CSR scatter of alpha_i w_im (Steps
//               5-6), dense rows (the adjoint's input), or the even reflection of
//               the lag quadrant (Step 2).  Writes frequency-major half spectra
//               through an LDS transpose so stores are whole cache lines.
//  k_cols       column pass over frequency-major half spectra (contiguous
//               columns): forward transform, product with the real filter
//               spectrum, inverse transform, keep the requested rows; variants
//               also accumulate sum_b G_b conj(C_b) (lag gradient), store the
//               forward real part (filter set-up), or invert a sum of partial
//               spectra.
//  k_rows_c2r   inverse transform back to real rows, two rows per complex line,
//               keeping the requested columns (optionally adding an image).
//
// Thread layout in all kernels: lane s (fastest, the transform's thread index)
// then line/column l; per-line LDS [l][n2][k1] with the n2 stride odd(N1) so the
// stage-A writes of consecutive lanes hit distinct banks.
#pragma once
#include "fft_args.h"
#include "fft_reg.h"
#include "matern_dev.h"
#include "philox_dev.h"

namespace krig {

__host__ __device__ constexpr int odd_up(int x) { return x | 1; }
__host__ __device__ constexpr int imax(int a, int b) { return a > b ? a : b; }

// Hide a value from the optimiser so address arithmetic and loads derived from it
// stay inside a loop (keeps loop-invariant values out of registers).
template <typename P>
__device__ __forceinline__ P opaque(P p) {
  asm volatile("" : "+s"(p));
  return p;
}
__device__ __forceinline__ int opaque_v(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <int N1, int N2> struct Geo {
  static constexpr int F = N1 * N2;
  static constexpr int NT = imax(N1, N2);
  static constexpr int ON1 = odd_up(N1);
  static constexpr int EX = N2 * ON1;                     // exchange slots per line
  static constexpr int ROWS = imax(EX, F + 2);            // row kernels: exchange or transpose
};

// LDS transposes [k][R] with the column rotated by k: lanes that differ in k (the
// fast lane index on one side of the transpose) fall on distinct banks, and a row
// stays a permutation of itself so the other side still reads whole rows.
__device__ __forceinline__ int rot(int k, int c, int R) { return k * R + (c + k) % R; }

__device__ __forceinline__ int window_dst(const Window& wd, int i) {
  if (i >= wd.a0 && i < wd.a0 + wd.na) return i - wd.a0;
  if (i >= wd.b0 && i < wd.b0 + wd.nb) return wd.na + i - wd.b0;
  return -1;
}

// ----------------------------------------------------------------------------------------
// the two register stages of a transform on one line, exchanged through LDS region
// L (stride ON1 between n2 rows).  On entry thread s < N2 holds v[n1] = x[N2 n1 + s];
// on exit thread s < N1 holds w[k2] = X[s + N1 k2].  DIR = -1 forward, +1 inverse.
// ----------------------------------------------------------------------------------------
template <typename TC, int N1, int N2, int DIR>
__device__ __forceinline__ void two_stage(cx<TC> (&v)[N1], cx<TC> (&w)[N2], int s, cx<TC>* L,
                                          const cx<TC>* twF) {
  using G = Geo<N1, N2>;
  if (s < N2) {
    DFT<N1, DIR, TC>::run(v);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      cx<TC> t = v[k1];
      if (k1 != 0 && s != 0) t = DIR < 0 ? cmul(t, twF[s * k1]) : cmulc(t, twF[s * k1]);
      L[s * G::ON1 + k1] = t;
    }
  }
  __syncthreads();
  if (s < N1) {
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) w[n2] = L[n2 * G::ON1 + s];
    DFT<N2, DIR, TC>::run(w);
  }
}

// inverse from the transposed order left by two_stage (thread s = k1 holds k2 =
// 0..N2-1); thread s < N2 ends with x[N2 n1 + s] in v[n1].
template <typename TC, int N1, int N2>
__device__ __forceinline__ void inv_from_t(cx<TC> (&w)[N2], int s, cx<TC>* L, const cx<TC>* twF,
                                           cx<TC> (&v)[N1]) {
  using G = Geo<N1, N2>;
  if (s < N1) {
    DFT<N2, 1, TC>::run(w);
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      cx<TC> t = w[n2];
      if (n2 != 0 && s != 0) t = cmulc(t, twF[n2 * s]);
      L[n2 * G::ON1 + s] = t;
    }
  }
  __syncthreads();
  if (s < N2) {
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[k1] = L[s * G::ON1 + k1];
    DFT<N1, 1, TC>::run(v);
  }
}

// ----------------------------------------------------------------------------------------
// row kernels: forward (real rows -> frequency-major half spectra)
// ----------------------------------------------------------------------------------------
enum { SRC_CSR = 0, SRC_DENSE = 1, SRC_LAG = 2, SRC_COV = 3 };

template <typename TC, typename TIN, typename TS, int N1, int N2, int SRC>
__global__ void __launch_bounds__(256) k_rows_r2c(RowsR2CArgs a) {
  using G = Geo<N1, N2>;
  extern __shared__ unsigned char smem_raw[];
  cx<TC>* lds = reinterpret_cast<cx<TC>*>(smem_raw);
  const int s = threadIdx.x % G::NT;
  const int l = threadIdx.x / G::NT;
  const int NL = a.NL;
  const int b = blockIdx.y;
  const int row0 = 2 * blockIdx.x * NL;
  const int ra = row0 + 2 * l, rb = ra + 1;
  const bool oka = ra < a.nrows, okb = rb < a.nrows;
  const cx<TC>* twF = reinterpret_cast<const cx<TC>*>(a.twF);
  cx<TC>* L = lds + (size_t)l * G::ROWS;

  cx<TC> v[N1];
  if (s < N2) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      const int c = N2 * n1 + s;
      TC xa = 0, xb = 0;
      if constexpr (SRC == SRC_CSR) {
        if (c < a.ncols) {
          const double* al = a.alpha + (int64_t)b * a.alpha_fs;
          if (oka) {
            const int q = ra * a.ncols + c;
            double acc = 0.0;
            for (int e = a.row_ptr[q]; e < a.row_ptr[q + 1]; ++e) acc += al[a.ent_site[e]] * a.ent_w[e];
            xa = (TC)acc;
          }
          if (okb) {
            const int q = rb * a.ncols + c;
            double acc = 0.0;
            for (int e = a.row_ptr[q]; e < a.row_ptr[q + 1]; ++e) acc += al[a.ent_site[e]] * a.ent_w[e];
            xb = (TC)acc;
          }
        }
      } else if constexpr (SRC == SRC_DENSE) {
        const int cc = c - a.coff;
        if (cc >= 0 && cc < a.ncols) {
          const TIN* d = reinterpret_cast<const TIN*>(a.dense) + (int64_t)b * a.dense_fs;
          if (oka) xa = (TC)d[(int64_t)ra * a.dense_ld + cc];
          if (okb) xb = (TC)d[(int64_t)rb * a.dense_ld + cc];
        }
      } else if constexpr (SRC == SRC_COV) {  // torus covariance with minimal-image lags
        const int F2 = G::F;
        MaternDev mt;
        mt.sigma2 = a.cov_sigma2;
        mt.rho = a.cov_rho;
        mt.tau2 = 0.0;
        mt.kind = a.cov_kind;
        const double hw = (double)(c < F2 - c ? c : F2 - c) * a.cov_dy;
        if (oka) {
          const double hu = (double)(ra < a.F1 - ra ? ra : a.F1 - ra) * a.cov_dx;
          xa = (TC)matern_cov(sqrt(hu * hu + hw * hw), mt);
        }
        if (okb) {
          const double hu = (double)(rb < a.F1 - rb ? rb : a.F1 - rb) * a.cov_dx;
          xb = (TC)matern_cov(sqrt(hu * hu + hw * hw), mt);
        }
      } else {  // SRC_LAG: embedding row r holds lag[min(r, F1-r)][min(c, F2-c)]
        const int F2 = G::F;
        const int dc = c < F2 - c ? c : F2 - c;
        if (dc < a.n2l) {
          if (oka) {
            const int dr = ra < a.F1 - ra ? ra : a.F1 - ra;
            if (dr < a.n1l) xa = (TC)a.lag[(int64_t)dr * a.n2l + dc];
          }
          if (okb) {
            const int dr = rb < a.F1 - rb ? rb : a.F1 - rb;
            if (dr < a.n1l) xb = (TC)a.lag[(int64_t)dr * a.n2l + dc];
          }
        }
      }
      v[n1] = mk<TC>(xa, xb);
    }
  }
  cx<TC> w[N2];
  two_stage<TC, N1, N2, -1>(v, w, s, L, twF);
  __syncthreads();
  // natural-order exchange to pair Z[k] with Z[F-k]
  if (s < N1) {
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) L[s + N1 * k2] = w[k2];
  }
  __syncthreads();
  constexpr int NK = (G::F / 2 + N1) / N1;  // k2 values with k = s + N1 k2 <= F/2 for some s
  cx<TC> xa[NK], xb[NK];
  if (s < N1) {
#pragma unroll
    for (int k2 = 0; k2 < NK; ++k2) {
      const int k = s + N1 * k2;
      const cx<TC> z = w[k2];
      const cx<TC> zc = L[(G::F - k) % G::F];
      // Xa = (Z[k] + conj Z[F-k]) / 2,  Xb = (Z[k] - conj Z[F-k]) / (2 i)
      xa[k2] = mk<TC>((TC)0.5 * (z.x + zc.x), (TC)0.5 * (z.y - zc.y));
      xb[k2] = mk<TC>((TC)0.5 * (z.y + zc.y), (TC)0.5 * (zc.x - z.x));
    }
  }
  __syncthreads();
  // transpose through LDS: T[k][2l + {0,1}] over the block, then row-contiguous stores
  cx<TC>* T = lds;
  const int R2 = 2 * NL;
  if (s < N1) {
#pragma unroll
    for (int k2 = 0; k2 < NK; ++k2) {
      const int k = s + N1 * k2;
      if (k < a.H2) {
        T[rot(k, 2 * l, R2)] = xa[k2];
        T[rot(k, 2 * l + 1, R2)] = xb[k2];
      }
    }
  }
  __syncthreads();
  cx<TS>* o = reinterpret_cast<cx<TS>*>(a.out) + (int64_t)b * a.out_fs;
  for (int idx = threadIdx.x; idx < a.H2 * R2; idx += blockDim.x) {
    const int rl = idx % R2, k = idx / R2;
    const int row = row0 + rl;
    if (row < a.nrows) o[(int64_t)k * a.out_ld + row] = ccast<TS>(T[rot(k, rl, R2)]);
  }
}

// ----------------------------------------------------------------------------------------
// column kernels (contiguous columns of frequency-major spectra)
// ----------------------------------------------------------------------------------------
template <typename TC, typename TS, int N1, int N2>
__device__ __forceinline__ void col_fwd(const cx<TS>* src, int in_off, int in_cnt, bool colok, int s,
                                        cx<TC>* L, const cx<TC>* twF, cx<TC> (&w)[N2]) {
  cx<TC> v[N1];
  if (s < N2) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      const int r = N2 * n1 + s - in_off;
      v[n1] = (colok && r >= 0 && r < in_cnt) ? ccast<TC>(src[r]) : mk<TC>(0, 0);
    }
  }
  two_stage<TC, N1, N2, -1>(v, w, s, L, twF);
}

enum { COL_CONV = 0, COL_CONV_DLAG = 1, COL_FWD_REAL = 2, COL_INV_SUM = 3, COL_CE = 4 };

template <typename TF, typename TI, typename TSI, typename TSO, int N1, int N2, int MODE>
__global__ void __launch_bounds__(256) k_cols(ColsArgs a) {
  using G = Geo<N1, N2>;
  using TC = TF;
  extern __shared__ unsigned char smem_raw[];
  const int NL = a.NL;
  const int s0 = threadIdx.x % G::NT;
  const int l0 = threadIdx.x / G::NT;
  const int col0 = blockIdx.x * NL + l0;
  const bool colok = col0 < a.H2;
  const cx<TC>* twF = reinterpret_cast<const cx<TC>*>(a.twF);
  cx<TC>* L = reinterpret_cast<cx<TC>*>(smem_raw) + (size_t)l0 * G::EX;
  const int s = s0, col = col0;

  if constexpr (MODE == COL_CONV) {
    const int b = blockIdx.y;
    const cx<TSI>* src = reinterpret_cast<const cx<TSI>*>(a.in) + (int64_t)b * a.in_fs + (int64_t)col * a.in_ld;
    cx<TI> wi[N2];
    {
      cx<TC> w[N2];
      col_fwd<TC, TSI, N1, N2>(src, a.in_off, a.in_cnt, colok, s, L, twF, w);
      if (s < N1 && colok) {
        const TF* f = reinterpret_cast<const TF*>(a.filt) + (int64_t)col * a.filt_ld;
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) w[k2] = cscale(w[k2], f[s + N1 * k2]);
      }
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) wi[k2] = ccast<TI>(w[k2]);
    }
    cx<TI>* LI = reinterpret_cast<cx<TI>*>(smem_raw) + (size_t)l0 * G::EX;
    cx<TI> v[N1];
    inv_from_t<TI, N1, N2>(wi, s, LI, reinterpret_cast<const cx<TI>*>(a.twI), v);
    if (s < N2 && colok) {
      cx<TSO>* dst = reinterpret_cast<cx<TSO>*>(a.out) + (int64_t)b * a.out_fs + (int64_t)col * a.out_ld;
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) {
        const int d = window_dst(a.rows, N2 * n1 + s);
        if (d >= 0) dst[d] = ccast<TSO>(v[n1]);
      }
    }
  } else if constexpr (MODE == COL_CONV_DLAG) {
    // blockIdx.y = group of G fields; partial spectrum of the group -> part[group]
    cx<TC> acc[N2];
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) acc[k2] = mk<TC>(0, 0);
    cx<TC>* stash = reinterpret_cast<cx<TC>*>(smem_raw) + (size_t)NL * G::EX + (size_t)l0 * G::F;
    const int b0 = blockIdx.y * a.G;
#pragma unroll 1
    for (int gi = 0; gi < a.G; ++gi) {
      const int b = b0 + gi;
      if (b >= a.B) break;  // uniform across the block
      twF = opaque(twF);
      // fresh copies of the lane indices each iteration: keeps per-lane address
      // arithmetic from being hoisted out of the field loop (register pressure)
      const int s = opaque_v(s0), col = opaque_v(col0);
      const cx<TSI>* srcc =
          reinterpret_cast<const cx<TSI>*>(a.in2) + (int64_t)b * a.in2_fs + (int64_t)col * a.in2_ld;
      const cx<TSI>* srcg = reinterpret_cast<const cx<TSI>*>(a.in) + (int64_t)b * a.in_fs + (int64_t)col * a.in_ld;
      __syncthreads();
      {
        // C-hat of this field: transform, then park it in this thread's stash slots
        cx<TC> wc[N2];
        col_fwd<TC, TSI, N1, N2>(srcc, a.in2_off, a.in2_cnt, colok, s, L, twF, wc);
        if (s < N1) {
#pragma unroll
          for (int k2 = 0; k2 < N2; ++k2) stash[k2 * N1 + s] = wc[k2];
        }
      }
      __syncthreads();
      cx<TC> wg[N2];
      col_fwd<TC, TSI, N1, N2>(srcg, a.in_off, a.in_cnt, colok, s, L, twF, wg);
      if (s < N1 && colok) {
        const TF* f = opaque(reinterpret_cast<const TF*>(a.filt)) + (int64_t)col * a.filt_ld;
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
          acc[k2] = acc[k2] + cmulc(wg[k2], stash[k2 * N1 + s]);
          wg[k2] = cscale(wg[k2], f[s + N1 * k2]);
        }
      }
      cx<TC> v[N1];
      inv_from_t<TC, N1, N2>(wg, s, L, twF, v);
      if (s < N2 && colok) {
        cx<TSO>* dst = reinterpret_cast<cx<TSO>*>(a.out) + (int64_t)b * a.out_fs + (int64_t)col * a.out_ld;
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
          const int d = window_dst(a.rows, N2 * n1 + s);
          if (d >= 0) dst[d] = ccast<TSO>(v[n1]);
        }
      }
    }
    if (s < N1 && colok) {
      cx<TSO>* p = reinterpret_cast<cx<TSO>*>(a.part) + (int64_t)blockIdx.y * a.part_fs + (int64_t)col * a.part_ld;
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) p[s + N1 * k2] = ccast<TSO>(acc[k2]);
    }
  } else if constexpr (MODE == COL_FWD_REAL) {
    // forward transform of the input columns; store Re(X) * scale (natural order)
    const int b = blockIdx.y;
    const cx<TSI>* src = reinterpret_cast<const cx<TSI>*>(a.in) + (int64_t)b * a.in_fs + (int64_t)col * a.in_ld;
    cx<TC> w[N2];
    col_fwd<TC, TSI, N1, N2>(src, a.in_off, a.in_cnt, colok, s, L, twF, w);
    if (s < N1 && colok) {
      TSO* dst = reinterpret_cast<TSO*>(a.out) + (int64_t)b * a.out_fs + (int64_t)col * a.out_ld;
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) dst[s + N1 * k2] = (TSO)(w[k2].x * (TC)a.scale);
    }
  } else if constexpr (MODE == COL_CE) {
    // sampler pass 1: column k2 (all ncol_full frequencies) of sqrt(Lambda/N) (xi1 + i xi2),
    // xi from Philox counter (k1 * ncol_full + k2, pair, STREAM_CE, 0); forward transform
    // over k1; keep rows [0, rows.na) -> out[pair][k2][r]
    const int pair = a.pair0 + blockIdx.y;
    const int kk2 = col < a.ncol_full - col ? col : a.ncol_full - col;  // Lambda is even
    const double* lam = reinterpret_cast<const double*>(a.filt) + (int64_t)kk2 * a.filt_ld;
    cx<TC> v[N1];
    if (s < N2) {
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) {
        const int k1 = N2 * n1 + s;
        cx<TC> z = mk<TC>(0, 0);
        if (colok) {
          u32x4 cn;
          cn.v[0] = (uint32_t)(k1 * a.ncol_full + col);
          cn.v[1] = (uint32_t)pair;
          cn.v[2] = STREAM_CE;
          cn.v[3] = 0;
          const u32x4 r = philox4x32_10(cn, a.key0, a.key1);
          double x0, x1;
          box_muller_f64(r.v[0], r.v[1], x0, x1);
          const double sl = lam[k1];
          z = mk<TC>((TC)(sl * x0), (TC)(sl * x1));
        }
        v[n1] = z;
      }
    }
    cx<TC> w[N2];
    two_stage<TC, N1, N2, -1>(v, w, s, L, twF);
    if (s < N1 && colok) {
      cx<TSO>* dst = reinterpret_cast<cx<TSO>*>(a.out) + (int64_t)blockIdx.y * a.out_fs + (int64_t)col * a.out_ld;
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const int d = window_dst(a.rows, s + N1 * k2);
        if (d >= 0) dst[d] = ccast<TSO>(w[k2]);
      }
    }
  } else {  // COL_INV_SUM: inverse transform of sum_g part[g] (natural order), keep rows
    const cx<TSI>* p = reinterpret_cast<const cx<TSI>*>(a.in) + (int64_t)col * a.in_ld;
    cx<TC> v[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) v[n1] = mk<TC>(0, 0);
    if (s < N2 && colok) {
      // partial g outermost: each round issues the N1 loads of one partial together;
      // every element is still summed in the order g = 0, 1, ...
      for (int g = 0; g < a.G; ++g) {
        const cx<TSI>* pg = p + (int64_t)g * a.in_fs + s;
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) v[n1] = v[n1] + ccast<TC>(pg[N2 * n1]);
      }
    }
    cx<TC> w[N2];
    two_stage<TC, N1, N2, 1>(v, w, s, L, twF);
    if (s < N1 && colok) {
      cx<TSO>* dst = reinterpret_cast<cx<TSO>*>(a.out) + (int64_t)col * a.out_ld;
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const int d = window_dst(a.rows, s + N1 * k2);
        if (d >= 0) dst[d] = ccast<TSO>(w[k2]);
      }
    }
  }
}

// ----------------------------------------------------------------------------------------
// row kernel: inverse (frequency-major half spectra -> real rows), two rows per line
// ----------------------------------------------------------------------------------------
template <typename TC, typename TS, typename TO, int N1, int N2>
__global__ void __launch_bounds__(256) k_rows_c2r(RowsC2RArgs a) {
  using G = Geo<N1, N2>;
  extern __shared__ unsigned char smem_raw[];
  cx<TC>* lds = reinterpret_cast<cx<TC>*>(smem_raw);
  const int s = threadIdx.x % G::NT;
  const int l = threadIdx.x / G::NT;
  const int NL = a.NL;
  const int b = blockIdx.y;
  const int row0 = 2 * blockIdx.x * NL;
  const int ra = row0 + 2 * l, rb = ra + 1;
  const bool oka = ra < a.nrows, okb = rb < a.nrows;
  const cx<TC>* twF = reinterpret_cast<const cx<TC>*>(a.twF);
  // row-contiguous loads of the block's 2 NL rows into T[k][rl]
  const int R2 = 2 * NL;
  cx<TC>* T = lds;
  const cx<TS>* in = reinterpret_cast<const cx<TS>*>(a.in) + (int64_t)b * a.in_fs;
  for (int idx = threadIdx.x; idx < a.H2 * R2; idx += blockDim.x) {
    const int rl = idx % R2, k = idx / R2;
    const int row = row0 + rl;
    T[rot(k, rl, R2)] = row < a.nrows ? ccast<TC>(in[(int64_t)k * a.in_ld + row]) : mk<TC>(0, 0);
  }
  __syncthreads();
  cx<TC> v[N1];
  if (s < N2) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      const int k = N2 * n1 + s;
      const bool lo = k < a.H2;
      const int kk = lo ? k : G::F - k;
      cx<TC> xa = T[rot(kk, 2 * l, R2)], xb = T[rot(kk, 2 * l + 1, R2)];
      if (kk == 0 || 2 * kk == G::F) { xa.y = 0; xb.y = 0; }  // DC / Nyquist are real
      if (!lo) { xa.y = -xa.y; xb.y = -xb.y; }
      v[n1] = mk<TC>(xa.x - xb.y, xa.y + xb.x);  // Xa + i Xb
    }
  }
  __syncthreads();
  cx<TC>* L = lds + (size_t)l * G::ROWS;
  cx<TC> w[N2];
  two_stage<TC, N1, N2, 1>(v, w, s, L, twF);
  if (s < N1) {
    TO* oa = reinterpret_cast<TO*>(a.out) + (int64_t)b * a.out_fs + (int64_t)ra * a.ldo;
    TO* ob = oa + a.ldo;
    const TO* ad = reinterpret_cast<const TO*>(a.add);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int c = s + N1 * k2;
      const int d = window_dst(a.cols, c);
      if (d >= 0) {
        TO va = (TO)w[k2].x, vb = (TO)w[k2].y;
        if (ad) {
          const TO* abase = ad + (int64_t)b * a.add_fs + (int64_t)(ra + a.add_r0) * a.add_ld + d + a.add_c0;
          if (oka) va += abase[0];
          if (okb) vb += abase[a.add_ld];
        }
        if (oka) oa[d] = va;
        if (okb) ob[d] = vb;
      }
    }
  }
}

// ----------------------------------------------------------------------------------------
// inverse rows of the compact correlation image with the sign images folded in:
// input rows (frequency-major) hold lags 0..n1l-1 then -(n1l-1)..-1 (compact row
// 2 n1l - 1 - u is lag -u); output row u < n1l, column w < n2l is
//   scale * sum over the sign images (+-u, +-w) of the correlation,
// each distinct image once (u = 0 or w = 0 has fewer).  The row fold is done on the
// input spectra (the row transform is linear), the column fold on the transformed
// line in LDS.
// ----------------------------------------------------------------------------------------
template <typename TC, typename TO, int N1, int N2>
__global__ void __launch_bounds__(256) k_rows_c2r_fold(RowsC2RArgs a) {
  using G = Geo<N1, N2>;
  extern __shared__ unsigned char smem_raw[];
  cx<TC>* lds = reinterpret_cast<cx<TC>*>(smem_raw);
  const int s = threadIdx.x % G::NT;
  const int l = threadIdx.x / G::NT;
  const int NL = a.NL;
  const int n1l = a.nrows, n2l = a.cols.na;
  const int row0 = 2 * blockIdx.x * NL;
  const int ra = row0 + 2 * l, rb = ra + 1;
  const cx<TC>* twF = reinterpret_cast<const cx<TC>*>(a.twF);
  const int R2 = 2 * NL;
  cx<TC>* T = lds;
  const cx<TC>* in = reinterpret_cast<const cx<TC>*>(a.in);
  for (int idx = threadIdx.x; idx < a.H2 * R2; idx += blockDim.x) {
    const int rl = idx % R2, k = idx / R2;
    const int u = row0 + rl;
    cx<TC> t = mk<TC>(0, 0);
    if (u < n1l) {
      t = in[(int64_t)k * a.in_ld + u];
      if (u > 0) t = t + in[(int64_t)k * a.in_ld + 2 * n1l - 1 - u];
    }
    T[rot(k, rl, R2)] = t;
  }
  __syncthreads();
  cx<TC> v[N1];
  if (s < N2) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      const int k = N2 * n1 + s;
      const bool lo = k < a.H2;
      const int kk = lo ? k : G::F - k;
      cx<TC> xa = T[rot(kk, 2 * l, R2)], xb = T[rot(kk, 2 * l + 1, R2)];
      if (kk == 0 || 2 * kk == G::F) { xa.y = 0; xb.y = 0; }  // DC / Nyquist are real
      if (!lo) { xa.y = -xa.y; xb.y = -xb.y; }
      v[n1] = mk<TC>(xa.x - xb.y, xa.y + xb.x);  // Xa + i Xb
    }
  }
  __syncthreads();
  cx<TC>* L = lds + (size_t)l * G::ROWS;
  cx<TC> w[N2];
  two_stage<TC, N1, N2, 1>(v, w, s, L, twF);
  __syncthreads();
  if (s < N1) {
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) L[s + N1 * k2] = w[k2];  // natural column order
  }
  __syncthreads();
  TO* oa = reinterpret_cast<TO*>(a.out) + (int64_t)ra * a.ldo;
  TO* ob = oa + a.ldo;
  const TC sc = (TC)a.scale;
  for (int c = s; c < n2l; c += G::NT) {
    cx<TC> y = L[c];
    if (c > 0) y = y + L[G::F - c];
    if (ra < n1l) oa[c] = (TO)(y.x * sc);
    if (rb < n1l) ob[c] = (TO)(y.y * sc);
  }
}

// ----------------------------------------------------------------------------------------
// sampler pass 2: complex forward transform of torus rows r < nrows (frequency-major
// input), keep columns < keep; real part -> realisation 2 pair, imaginary -> 2 pair + 1
// ----------------------------------------------------------------------------------------
template <typename TC, typename TS, typename TO, int N1, int N2>
__global__ void __launch_bounds__(256) k_rows_ce(RowsCEArgs a) {
  using G = Geo<N1, N2>;
  extern __shared__ unsigned char smem_raw[];
  cx<TC>* lds = reinterpret_cast<cx<TC>*>(smem_raw);
  const int s = threadIdx.x % G::NT;
  const int l = threadIdx.x / G::NT;
  const int NL = a.NL;
  const int pair = a.pair0 + blockIdx.y;
  const int row0 = blockIdx.x * NL;
  const int row = row0 + l;
  const cx<TC>* twF = reinterpret_cast<const cx<TC>*>(a.twF);
  const cx<TS>* in = reinterpret_cast<const cx<TS>*>(a.in) + (int64_t)blockIdx.y * a.in_fs;
  cx<TC>* T = lds;  // [k][l]
  for (int idx = threadIdx.x; idx < G::F * NL; idx += blockDim.x) {
    const int rl = idx % NL, k = idx / NL;
    const int r = row0 + rl;
    T[rot(k, rl, NL)] = r < a.nrows ? ccast<TC>(in[(int64_t)k * a.in_ld + r]) : mk<TC>(0, 0);
  }
  __syncthreads();
  cx<TC> v[N1];
  if (s < N2) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) v[n1] = T[rot(N2 * n1 + s, l, NL)];
  }
  __syncthreads();
  cx<TC>* L = lds + (size_t)l * G::EX;
  cx<TC> w[N2];
  two_stage<TC, N1, N2, -1>(v, w, s, L, twF);
  if (s < N1 && row < a.nrows) {
    const int re = 2 * pair, im = 2 * pair + 1;
    TO* o1 = reinterpret_cast<TO*>(a.out) + (int64_t)re * a.out_fs + (int64_t)row * a.ldo;
    TO* o2 = reinterpret_cast<TO*>(a.out) + (int64_t)im * a.out_fs + (int64_t)row * a.ldo;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int c = s + N1 * k2;
      if (c < a.keep) {
        if (re < a.R) o1[c] = (TO)w[k2].x;
        if (im < a.R) o2[c] = (TO)w[k2].y;
      }
    }
  }
}

// ----------------------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------------------
template <typename TC, typename TIN, typename TS, int N1, int N2, int SRC>
hipError_t launch_rows_r2c(const RowsR2CArgs& a, int B, hipStream_t st) {
  const int npairs = (a.nrows + 1) / 2;
  dim3 grid((npairs + a.NL - 1) / a.NL, B);
  dim3 block(Geo<N1, N2>::NT * a.NL);
  const size_t sh = rows_lds(N1, N2, a.NL, sizeof(cx<TC>));
  k_rows_r2c<TC, TIN, TS, N1, N2, SRC><<<grid, block, sh, st>>>(a);
  return hipGetLastError();
}

template <typename TF, typename TI, typename TSI, typename TSO, int N1, int N2, int MODE>
hipError_t launch_cols(const ColsArgs& a, int nblk_y, hipStream_t st) {
  dim3 grid((a.H2 + a.NL - 1) / a.NL, nblk_y);
  dim3 block(Geo<N1, N2>::NT * a.NL);
  const size_t sh = cols_lds(N1, N2, a.NL, sizeof(cx<TF>), MODE == COL_CONV_DLAG);
  k_cols<TF, TI, TSI, TSO, N1, N2, MODE><<<grid, block, sh, st>>>(a);
  return hipGetLastError();
}

template <typename TC, typename TS, typename TO, int N1, int N2>
hipError_t launch_rows_c2r(const RowsC2RArgs& a, int B, hipStream_t st) {
  const int npairs = (a.nrows + 1) / 2;
  dim3 grid((npairs + a.NL - 1) / a.NL, B);
  dim3 block(Geo<N1, N2>::NT * a.NL);
  const size_t sh = rows_lds(N1, N2, a.NL, sizeof(cx<TC>));
  k_rows_c2r<TC, TS, TO, N1, N2><<<grid, block, sh, st>>>(a);
  return hipGetLastError();
}

template <typename TC, typename TO, int N1, int N2>
hipError_t launch_rows_c2r_fold(const RowsC2RArgs& a, int B, hipStream_t st) {
  const int npairs = (a.nrows + 1) / 2;
  dim3 grid((npairs + a.NL - 1) / a.NL, 1);
  dim3 block(Geo<N1, N2>::NT * a.NL);
  const size_t sh = rows_lds(N1, N2, a.NL, sizeof(cx<TC>));
  (void)B;
  k_rows_c2r_fold<TC, TO, N1, N2><<<grid, block, sh, st>>>(a);
  return hipGetLastError();
}

template <typename TC, typename TS, typename TO, int N1, int N2>
hipError_t launch_rows_ce(const RowsCEArgs& a, int npairs, hipStream_t st) {
  dim3 grid((a.nrows + a.NL - 1) / a.NL, npairs);
  dim3 block(Geo<N1, N2>::NT * a.NL);
  const size_t sh = ce_rows_lds(N1, N2, a.NL, sizeof(cx<TC>));
  k_rows_ce<TC, TS, TO, N1, N2><<<grid, block, sh, st>>>(a);
  return hipGetLastError();
}

template <int N1, int N2>
FftEntry make_fft_entry() {
  FftEntry e;
  e.F = N1 * N2;
  e.N1 = N1;
  e.N2 = N2;
  FftSet& k = e.k;
  k.r2c_csr = launch_rows_r2c<double, double, double, N1, N2, SRC_CSR>;
  k.r2c_dense_f32 = launch_rows_r2c<double, float, double, N1, N2, SRC_DENSE>;
  k.r2c_dense_f64 = launch_rows_r2c<double, double, double, N1, N2, SRC_DENSE>;
  k.r2c_lag = launch_rows_r2c<double, double, double, N1, N2, SRC_LAG>;
  k.conv_mixed = launch_cols<double, float, double, float, N1, N2, COL_CONV>;
  k.conv64 = launch_cols<double, double, double, double, N1, N2, COL_CONV>;
  k.conv_dlag64 = launch_cols<double, double, double, double, N1, N2, COL_CONV_DLAG>;
  k.fwd_real64 = launch_cols<double, double, double, double, N1, N2, COL_FWD_REAL>;
  k.inv_sum64 = launch_cols<double, double, double, double, N1, N2, COL_INV_SUM>;
  k.c2r32 = launch_rows_c2r<float, float, float, N1, N2>;
  k.c2r64 = launch_rows_c2r<double, double, double, N1, N2>;
  k.c2r_fold32 = launch_rows_c2r_fold<double, float, N1, N2>;
  k.c2r_fold64 = launch_rows_c2r_fold<double, double, N1, N2>;
  k.r2c_cov = launch_rows_r2c<double, double, double, N1, N2, SRC_COV>;
  k.ce_cols32 = launch_cols<float, float, float, float, N1, N2, COL_CE>;
  k.ce_cols64 = launch_cols<double, double, double, double, N1, N2, COL_CE>;
  k.ce_rows32 = launch_rows_ce<float, float, float, N1, N2>;
  k.ce_rows64 = launch_rows_ce<double, double, double, N1, N2>;
  return e;
}

}  // namespace krig

#define KRIG_FFT_SIZE(N1, N2)                                                 \
  namespace krig {                                                            \
  void register_fft_##N1##x##N2() { register_fft(make_fft_entry<N1, N2>()); } \
  }
