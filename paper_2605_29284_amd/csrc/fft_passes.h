// FFT pass kernels for the circulant-embedded convolution (Step 7) and its adjoint,
// and the circulant-embedding sampler.  Included by one generated translation unit
// per transform length F = R1 * R2 * R3 (factorisation and register layouts: see
// fft_args.h).
//
// Roles (TC/TF/TI = arithmetic precision; TS, TO and the column passes' Stor set =
// storage forms, see spec_io.h):
//  k_rows_r2c   forward transform of real rows, two rows per complex line
//               ("two-for-one"); sources: the CSR scatter of alpha_i w_im (Steps
//               5-6), dense rows (the adjoint's input), the even reflection of the
//               lag quadrant (Step 2), or the covariance on the sampler's torus.
//               Writes frequency-major half spectra through an LDS transpose so
//               stores are whole cache lines.
//  k_cols       column pass over frequency-major half spectra (contiguous
//               columns): forward transform, product with the real filter
//               spectrum, inverse transform, keep the requested rows; variants
//               also accumulate sum_b G_b conj(C_b) (lag gradient), store the
//               forward real part (filter set-up), invert a sum of partial
//               spectra, or draw the sampler's noise.
//  k_rows_c2r   inverse transform back to real rows, two rows per complex line,
//               keeping the requested columns (optionally adding an image); a
//               folded form for the lag gradient.
//  k_rows_ce    the sampler's complex row transforms.
//
// Thread layout in all kernels: lane s (fastest, the transform's thread index, NT
// per line) then line/column l.  Every transform begins with a block barrier, since
// a line may span two waves and reuses the LDS of the previous step.
#pragma once
#include <type_traits>

#include "fft_args.h"
#include "fft_reg.h"
#include "matern_dev.h"
#include "philox_dev.h"
#include "spec_io.h"

namespace krig {

template <int R1_, int R2_, int R3_> struct Geo {
  static constexpr FftGeo g = fft_geo(R1_, R2_, R3_);
  static constexpr int R1 = R1_, R2 = R2_, R3 = R3_;
  static constexpr int F = g.F, M = g.M, NIN = g.NIN, TIN = g.TIN, NOUT = g.NOUT, TOUT = g.TOUT, T2 = g.T2;
  static constexpr int NT = g.NT, ON2 = g.ON2, RS = g.RS, P1 = g.P1, EX = g.EX, ROWS = g.ROWS;
  static constexpr bool THREE = R1_ > 1;
};

// Hide a value from the optimiser so address arithmetic derived from it stays
// inside a loop (keeps loop-invariant values out of registers).
template <typename P>
__device__ __forceinline__ P opaque(P p) {
  asm volatile("" : "+s"(p));
  return p;
}
__device__ __forceinline__ int opaque_v(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// a * tw (DIR < 0) or a * conj(tw) (DIR > 0)
template <int DIR, typename T>
__device__ __forceinline__ cx<T> twm(cx<T> a, cx<T> tw) {
  return DIR < 0 ? cmul(a, tw) : cmulc(a, tw);
}

// Three-pass row kernels with an outer radix of at most 8, a middle one of at most 12
// and an inner one of at most 9 hold about 100 VGPRs; capped at 96 (five waves per
// SIMD) they still need no scratch, and six 3-wave blocks (27 KB of LDS each at length
// 768) then share a CU, so a pass over ~1,400 row blocks (16 fields) runs in one round
// instead of 1.1.  Other forms keep the default: the cap would make them spill.
template <int R1, int R2, int R3> struct RowCap {
  static constexpr int waves = (R1 > 1 && R1 <= 8 && R2 <= 12 && R3 <= 9) ? 5 : 1;
};
#define KRIG_ROW_KERNEL \
  __global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RowCap<R1, R2, R3>::waves)))

// LDS transposes [k][R].  A wave's 16-byte LDS accesses go eight lanes at a time over
// 16 bank groups of 16 bytes.  Eight lanes with consecutive k (one side of the
// transpose) fall on distinct groups when R is not a multiple of 4.  For R = 4, 8, 16,
// ... the columns of row k are rotated by floor(k / p), p = 16 / R (1 from R = 16 on):
// rows k and k + p, which start in the same group, are then shifted one group apart.
// Other multiples of 4 get a padded pitch (tpitch).  Lanes with consecutive c (the other
// side) stay within one row or run into the next.
__device__ __forceinline__ int tpos(int k, int c, int R) {
  if ((R & 3) != 0 || (R & (R - 1)) != 0) return k * tpitch(R) + c;
  const int sh = R >= 16 ? 0 : (R == 8 ? 1 : 2);
  return k * R + ((c + (k >> sh)) & (R - 1));
}

// The elements idx = tid, tid + NT NL, tid + 2 NT NL, ... of a [k][2 NL] transpose as
// (k, rl) = (idx / (2 NL), idx mod 2 NL), stepped without a division: a step adds
// NT NL = (NT / 2) 2 NL + (NT mod 2) NL.
template <int NT> struct TWalk {
  int k, rl;
  const int nl;
  __device__ __forceinline__ TWalk(int tid, int NL) : k(tid / (2 * NL)), rl(tid % (2 * NL)), nl(NL) {}
  __device__ __forceinline__ void next() {
    k += NT / 2;
    if constexpr (NT % 2 != 0) {
      rl += nl;
      if (rl >= 2 * nl) { rl -= 2 * nl; ++k; }
    }
  }
};

// Workgroups go to the 8 XCDs (each with its own L2) round-robin by linear block id.
// xcd_block maps the hardware id to a logical id so that each XCD runs one contiguous
// range of logical blocks; blocks that share cache lines (neighbouring row blocks of a
// frequency-major spectrum) or a filter column (the fields of one column) then share
// an L2 instead of fetching the same lines once per XCD.
constexpr int KRIG_XCDS = 8;
__device__ __forceinline__ int xcd_block(int bid, int nb) {
  const int per = nb / KRIG_XCDS, rem = nb % KRIG_XCDS;
  const int x = bid % KRIG_XCDS, k = bid / KRIG_XCDS;
  return x * per + (x < rem ? x : rem) + k;
}
// logical (bx, by) of this block: rows kernels order bx fastest (row blocks of a field
// contiguous), column kernels order by fastest (the fields of a column contiguous)
template <bool Y_FAST>
__device__ __forceinline__ void logical_block(int& bx, int& by) {
  const int lb = xcd_block(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  if (Y_FAST) {
    by = lb % gridDim.y;
    bx = lb / gridDim.y;
  } else {
    bx = lb % gridDim.x;
    by = lb / gridDim.x;
  }
}

__device__ __forceinline__ int window_dst(const Window& wd, int i) {
  if (i >= wd.a0 && i < wd.a0 + wd.na) return i - wd.a0;
  if (i >= wd.b0 && i < wd.b0 + wd.nb) return wd.na + i - wd.b0;
  return -1;
}

// ----------------------------------------------------------------------------------------
// Pass twiddles.  Each thread loads a few base powers b of W = exp(-2 pi i / F) once,
// before its first transform, and forms the powers a pass needs by repeated
// multiplication (loading them inside a pass put a memory latency after every barrier):
//   f1 = W^t (pass 1), f2 = W^(R1 (t mod R3)) (pass 2); for the inverse from the output
//   layout also i3 = W^(R1 floor(t / R1)), i4a = W^(floor(t / R3) (t mod R3)) and
//   i4b = W^(R3 floor(t / R3)).
// A table entry b = W^j (1 + d) carries a rounding d of about 2^-54, and b^k carries k d,
// which for k up to 15 outweighed the rounding of the products and doubled the FP64
// transform error.  The table stores d (FP32) after its F entries; every fourth step the
// running power is multiplied by (1 + 4 d) (first order in d), so no power carries more
// than 3 d.  Measured on the convolution sweep this matches direct table loads.
// ----------------------------------------------------------------------------------------
template <typename TC> struct TwB {
  cx<TC> f1, f2, i3, i4a, i4b;
  cx<float> d1, d2, d3, d4;  // relative rounding of f1, f2, i3, i4b
};

// Threads outside a pass's range read entry 0, which is exactly 1 (d = 0).
template <typename TC, int R1, int R2, int R3, bool INV>
__device__ __forceinline__ TwB<TC> tw_bases(const cx<TC>* tw, int t) {
  using G = Geo<R1, R2, R3>;
  const cx<float>* td = reinterpret_cast<const cx<float>*>(tw + G::F);
  const int j1 = (G::THREE && t < G::TIN) ? t : 0;
  const int j2 = t < G::T2 ? R1 * (t % R3) : 0;
  const int j3 = (INV && t < G::TOUT) ? R1 * (t / R1) : 0;
  const int j4 = (INV && G::THREE && t < G::T2) ? R3 * (t / R3) : 0;
  TwB<TC> b;
  b.f1 = tw[j1];
  b.f2 = tw[j2];
  b.i3 = tw[j3];
  b.i4a = tw[(INV && G::THREE && t < G::T2) ? (t / R3) * (t % R3) : 0];
  b.i4b = tw[j4];
  b.d1 = td[j1];
  b.d2 = td[j2];
  b.d3 = td[j3];
  b.d4 = td[j4];
  return b;
}

// p (1 + k d): removes the rounding d of k table-entry factors from the product p.
template <typename TC>
__device__ __forceinline__ cx<TC> tw_fix(cx<TC> p, cx<float> d, int k) {
  const TC er = (TC)(d.x * (float)k), ei = (TC)(d.y * (float)k);
  return mk<TC>(fma(p.x, er, fma(-p.y, ei, p.x)), fma(p.x, ei, fma(p.y, er, p.y)));
}

// ----------------------------------------------------------------------------------------
// One transform per line, input layout -> output layout (DIR = -1 forward, +1
// inverse, unnormalised).  L: the line's EX LDS slots; tw: exp(-2 pi i j / F), j < F.
//  pass 1 (R1 > 1): thread m < M: DFT_R1 over j of x[m + M j], times W_F^(m k1),
//                   to L[k1 P1 + m]
//  pass 2: thread (k1, s), t = k1 R3 + s: DFT_R2 over n1 of z_k1[R3 n1 + s], times
//          W_M^(s s'), to L[k1 RS + s ON2 + s']
//  pass 3: thread (k1, s'), t = s' R1 + k1: DFT_R3 over s -> X[k1 + R1 s' + R1 R2 k2]
//          = X[t + TOUT k2]
// ----------------------------------------------------------------------------------------
template <typename TC, int R1, int R2, int R3, int DIR>
__device__ __forceinline__ void xf_fwd(cx<TC> (&v)[(Geo<R1, R2, R3>::NIN)], cx<TC> (&w)[R3], int t, cx<TC>* L,
                                       const TwB<TC>& tb) {
  using G = Geo<R1, R2, R3>;
  __syncthreads();
  cx<TC> u[R2];
  if constexpr (G::THREE) {
    if (t < G::TIN) {
      DFT<R1, DIR, TC>::run(v);
      cx<TC> wk = tb.f1;  // W^(t k1)
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) {
        cx<TC> a = v[k1];
        if (k1 != 0) {
          if (k1 > 1) wk = cmul(wk, tb.f1);
          if (k1 % 4 == 0) wk = tw_fix(wk, tb.d1, 4);
          a = twm<DIR>(a, wk);
        }
        L[k1 * G::P1 + t] = a;
      }
    }
    __syncthreads();
    if (t < G::T2) {
      const int k1 = t / R3, s = t % R3;
#pragma unroll
      for (int n1 = 0; n1 < R2; ++n1) u[n1] = L[k1 * G::P1 + R3 * n1 + s];
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int n1 = 0; n1 < R2; ++n1) u[n1] = v[n1];
  }
  if (t < G::T2) {
    const int k1 = t / R3, s = t % R3;
    DFT<R2, DIR, TC>::run(u);
    cx<TC>* Lk = L + k1 * G::RS;
    cx<TC> wq = tb.f2;  // W^(R1 s q)
#pragma unroll
    for (int q = 0; q < R2; ++q) {
      cx<TC> a = u[q];
      if (q != 0) {
        if (q > 1) wq = cmul(wq, tb.f2);
        if (q % 4 == 0) wq = tw_fix(wq, tb.d2, 4);
        a = twm<DIR>(a, wq);
      }
      Lk[s * G::ON2 + q] = a;
    }
  }
  __syncthreads();
  if (t < G::TOUT) {
    const int k1 = t % R1, sp = t / R1;
    const cx<TC>* Lk = L + k1 * G::RS;
#pragma unroll
    for (int n2 = 0; n2 < R3; ++n2) w[n2] = Lk[n2 * G::ON2 + sp];
    DFT<R3, DIR, TC>::run(w);
  }
}

// Inverse transform from the output layout (thread t < TOUT holds X[t + TOUT k2])
// back to the input layout (thread t < TIN ends with x[t + TIN j] in v[j]): the
// passes of xf_fwd in reverse with conjugate twiddles.
template <typename TC, int R1, int R2, int R3>
__device__ __forceinline__ void xf_inv(cx<TC> (&w)[R3], int t, cx<TC>* L, const TwB<TC>& tb,
                                       cx<TC> (&v)[(Geo<R1, R2, R3>::NIN)]) {
  using G = Geo<R1, R2, R3>;
  __syncthreads();
  if (t < G::TOUT) {
    const int k1 = t % R1, sp = t / R1;
    DFT<R3, 1, TC>::run(w);
    cx<TC>* Lk = L + k1 * G::RS;
    cx<TC> wn = tb.i3;  // W^(R1 sp n2)
#pragma unroll
    for (int n2 = 0; n2 < R3; ++n2) {
      cx<TC> a = w[n2];
      if (n2 != 0) {
        if (n2 > 1) wn = cmul(wn, tb.i3);
        if (n2 % 4 == 0) wn = tw_fix(wn, tb.d3, 4);
        a = cmulc(a, wn);
      }
      Lk[n2 * G::ON2 + sp] = a;
    }
  }
  __syncthreads();
  cx<TC> u[R2];
  if (t < G::T2) {
    const int k1 = t / R3, n2 = t % R3;
#pragma unroll
    for (int q = 0; q < R2; ++q) u[q] = L[k1 * G::RS + n2 * G::ON2 + q];
  }
  if constexpr (G::THREE) {
    __syncthreads();
    if (t < G::T2) {
      const int k1 = t / R3, n2 = t % R3;
      DFT<R2, 1, TC>::run(u);
      cx<TC> wm = tb.i4a;  // W^(m k1), m = R3 n1 + n2
#pragma unroll
      for (int n1 = 0; n1 < R2; ++n1) {
        const int m = R3 * n1 + n2;
        if (n1 > 0) wm = cmul(wm, tb.i4b);
        if (n1 > 0 && n1 % 4 == 0) wm = tw_fix(wm, tb.d4, 4);
        L[k1 * G::P1 + m] = cmulc(u[n1], wm);
      }
    }
    __syncthreads();
    if (t < G::TIN) {
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) v[k1] = L[k1 * G::P1 + t];
      DFT<R1, 1, TC>::run(v);
    }
  } else {
    if (t < G::T2) {
      DFT<R2, 1, TC>::run(u);
#pragma unroll
      for (int n1 = 0; n1 < R2; ++n1) v[n1] = u[n1];
    }
  }
}

// ----------------------------------------------------------------------------------------
// row kernels: forward (real rows -> frequency-major half spectra)
// ----------------------------------------------------------------------------------------
enum { SRC_CSR = 0, SRC_DENSE = 1, SRC_LAG = 2, SRC_COV = 3, SRC_CENTER = 4, SRC_DELTA = 5 };

template <typename TC, typename TIN, typename TS, int R1, int R2, int R3, int SRC>
KRIG_ROW_KERNEL k_rows_r2c(RowsR2CArgs a) {
  int bx, by;
  logical_block<false>(bx, by);
  using G = Geo<R1, R2, R3>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<TC>* lds = reinterpret_cast<cx<TC>*>(smem_raw);
  const int s = threadIdx.x % G::NT;
  const int l = threadIdx.x / G::NT;
  const int NL = a.NL;
  const int b = by;
  const int row0 = 2 * bx * NL;
  const int ra = row0 + 2 * l, rb = ra + 1;
  const bool oka = ra < a.nrows, okb = rb < a.nrows;
  const cx<TC>* twF = reinterpret_cast<const cx<TC>*>(a.twF);
  const TwB<TC> tb = tw_bases<TC, R1, R2, R3, false>(twF, s);
  cx<TC>* L = lds + (size_t)l * G::ROWS;

  cx<TC> v[G::NIN];
  // CSR scatter (Steps 5-6): node (r, c) = sum over its segment of alpha[site] * w, in
  // segment order.  For each of the line's two rows the loads of its NIN nodes go out
  // in three batches (segment bounds, first entries, their alphas) instead of one
  // dependent chain per node; later entries of a segment (rare) follow in a loop.
  double sc[2][G::NIN];
  if constexpr (SRC == SRC_CSR) {
    if (s < G::TIN) {
      const double* al = a.alpha + (int64_t)b * a.alpha_fs;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int rr = h ? rb : ra;
        const bool okr = h ? okb : oka;
        int e0[G::NIN], e1[G::NIN];
#pragma unroll
        for (int j = 0; j < G::NIN; ++j) {
          const int c = G::TIN * j + s;
          const bool ok = okr && c < a.ncols;
          const int q = rr * a.ncols + c;
          e0[j] = ok ? a.row_ptr[q] : 0;
          e1[j] = ok ? a.row_ptr[q + 1] : 0;
        }
        int site[G::NIN];
        double w0[G::NIN];
#pragma unroll
        for (int j = 0; j < G::NIN; ++j) {
          const bool has = e0[j] < e1[j];
          site[j] = has ? a.ent_site[e0[j]] : 0;
          w0[j] = has ? a.ent_w[e0[j]] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < G::NIN; ++j) {
          sc[h][j] = 0.0;
          if (e0[j] < e1[j]) sc[h][j] += al[site[j]] * w0[j];
        }
#pragma unroll
        for (int j = 0; j < G::NIN; ++j)
          for (int e = e0[j] + 1; e < e1[j]; ++e) sc[h][j] += al[a.ent_site[e]] * a.ent_w[e];
      }
    }
  }
  if (s < G::TIN) {
#pragma unroll
    for (int j = 0; j < G::NIN; ++j) {
      const int c = G::TIN * j + s;
      TC xa = 0, xb = 0;
      if constexpr (SRC == SRC_CSR) {
        xa = (TC)sc[0][j];
        xb = (TC)sc[1][j];
      } else if constexpr (SRC == SRC_DENSE) {
        const int cc = c - a.coff;
        if (cc >= 0 && cc < a.ncols) {
          const TIN* d = reinterpret_cast<const TIN*>(a.dense) + (int64_t)b * a.dense_fs;
          if (oka) xa = (TC)d[(int64_t)ra * a.dense_ld + cc];
          if (okb) xb = (TC)d[(int64_t)rb * a.dense_ld + cc];
        }
      } else if constexpr (SRC == SRC_CENTER) {  // covariance about the torus centre, plain coordinates
        const int F2 = G::F;
        MaternDev mt;
        mt.sigma2 = a.cov_sigma2;
        mt.rho = a.cov_rho;
        mt.tau2 = 0.0;
        mt.kind = a.cov_kind;
        const double hw = (double)(c - F2 / 2) * a.cov_dy;
        if (oka) {
          const double hu = (double)(ra - a.F1 / 2) * a.cov_dx;
          xa = (TC)matern_cov(sqrt(hu * hu + hw * hw), mt);
        }
        if (okb) {
          const double hu = (double)(rb - a.F1 / 2) * a.cov_dx;
          xb = (TC)matern_cov(sqrt(hu * hu + hw * hw), mt);
        }
      } else if constexpr (SRC == SRC_DELTA) {  // indicator of the torus centre
        const bool cc = c == G::F / 2;
        xa = (TC)((cc && oka && ra == a.F1 / 2) ? 1 : 0);
        xb = (TC)((cc && okb && rb == a.F1 / 2) ? 1 : 0);
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
      v[j] = mk<TC>(xa, xb);
    }
  }
  cx<TC> w[G::NOUT];
  xf_fwd<TC, R1, R2, R3, -1>(v, w, s, L, tb);
  __syncthreads();
  // natural-order exchange to pair Z[k] with Z[F-k]
  if (s < G::TOUT) {
#pragma unroll
    for (int k2 = 0; k2 < G::NOUT; ++k2) L[s + G::TOUT * k2] = w[k2];
  }
  __syncthreads();
  constexpr int NK = (G::F / 2 + G::TOUT) / G::TOUT;  // k2 with k = s + TOUT k2 <= F/2 for some s
  cx<TC> xa[NK], xb[NK];
  if (s < G::TOUT) {
#pragma unroll
    for (int k2 = 0; k2 < NK; ++k2) {
      const int k = s + G::TOUT * k2;
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
  const int R2b = 2 * NL;
  if (s < G::TOUT) {
#pragma unroll
    for (int k2 = 0; k2 < NK; ++k2) {
      const int k = s + G::TOUT * k2;
      if (k < a.H2) {
        T[tpos(k, 2 * l, R2b)] = xa[k2];
        T[tpos(k, 2 * l + 1, R2b)] = xb[k2];
      }
    }
  }
  __syncthreads();
  const Spec<TS> o = Spec<TS>::field(a.out, a.out_fs, b);
  // element idx = k R2b + rl of the transpose goes to thread idx mod blockDim (NT NL)
  for (TWalk<G::NT> e(threadIdx.x, NL); e.k < a.H2; e.next()) {
    const int row = row0 + e.rl;
    if (row < a.nrows) o.st((int64_t)e.k * a.out_ld + row, T[tpos(e.k, e.rl, R2b)]);
  }
}

// ----------------------------------------------------------------------------------------
// column kernels (contiguous columns of frequency-major spectra)
// ----------------------------------------------------------------------------------------
template <typename TC, typename TS, int R1, int R2, int R3>
__device__ __forceinline__ void col_fwd(const Spec<TS> src, int in_off, int in_cnt, bool colok, int s,
                                        cx<TC>* L, const TwB<TC>& tb, cx<TC> (&w)[R3]) {
  using G = Geo<R1, R2, R3>;
  cx<TC> v[G::NIN];
  if (s < G::TIN) {
#pragma unroll
    for (int j = 0; j < G::NIN; ++j) {
      const int r = G::TIN * j + s - in_off;
      v[j] = (colok && r >= 0 && r < in_cnt) ? src.template ld<TC>(r) : mk<TC>(0, 0);
    }
  }
  xf_fwd<TC, R1, R2, R3, -1>(v, w, s, L, tb);
}

enum { COL_CONV = 0, COL_CONV_DLAG = 1, COL_FWD_REAL = 2, COL_INV_SUM = 3, COL_CE = 4 };

// The lag-gradient column pass (two forward transforms and an inverse per line) of the
// same forms needs just over 168 VGPRs.  Capped at three waves per SIMD it spills a few
// dozen bytes per lane and still runs faster than uncapped at two waves; a four-wave cap
// (over 200 bytes of scratch) runs at half speed.  The plain convolution pass keeps the
// default (four waves): a five-wave cap made it spill and run slower.
template <int R1, int R2, int R3, int MODE> struct ColCap {
  static constexpr int waves = (MODE == COL_CONV_DLAG && RowCap<R1, R2, R3>::waves > 1) ? 3 : 1;
};

template <typename TF, typename TI, typename ST, int R1, int R2, int R3, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ColCap<R1, R2, R3, MODE>::waves)))
k_cols(ColsArgs a) {
  using TSI = typename ST::in;
  using TSO = typename ST::out;
  int bx, by;
  logical_block<true>(bx, by);
  using G = Geo<R1, R2, R3>;
  using TC = TF;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int NL = a.NL;
  const int s = threadIdx.x % G::NT;
  const int l0 = threadIdx.x / G::NT;
  const int col = bx * NL + l0;
  const bool colok = col < a.H2;
  const cx<TC>* twF = reinterpret_cast<const cx<TC>*>(a.twF);
  static_assert(std::is_same<TI, TF>::value, "one arithmetic type per column pass");
  const TwB<TC> tb = tw_bases<TC, R1, R2, R3, (MODE == COL_CONV || MODE == COL_CONV_DLAG)>(twF, s);
  cx<TC>* L = reinterpret_cast<cx<TC>*>(smem_raw) + (size_t)l0 * G::EX;

  if constexpr (MODE == COL_CONV) {
    const int b = by;
    const Spec<TSI> src = Spec<TSI>::field(a.in, a.in_fs, b).at((int64_t)col * a.in_ld);
    // the filter values this thread needs, loaded before the transform hides their latency
    TF fv[R3];
    {
      const TF* f = reinterpret_cast<const TF*>(a.filt) + (int64_t)(colok ? col : 0) * a.filt_ld;
#pragma unroll
      for (int k2 = 0; k2 < R3; ++k2) fv[k2] = (s < G::TOUT && colok) ? f[s + G::TOUT * k2] : (TF)0;
    }
    cx<TI> wi[R3];
    {
      cx<TC> w[R3];
      col_fwd<TC, TSI, R1, R2, R3>(src, a.in_off, a.in_cnt, colok, s, L, tb, w);
      if (s < G::TOUT && colok) {
#pragma unroll
        for (int k2 = 0; k2 < R3; ++k2) w[k2] = cscale(w[k2], fv[k2]);
      }
#pragma unroll
      for (int k2 = 0; k2 < R3; ++k2) wi[k2] = ccast<TI>(w[k2]);
    }
    cx<TI>* LI = reinterpret_cast<cx<TI>*>(smem_raw) + (size_t)l0 * G::EX;
    cx<TI> v[G::NIN];
    xf_inv<TI, R1, R2, R3>(wi, s, LI, tb, v);
    if (s < G::TIN && colok) {
      const Spec<TSO> dst = Spec<TSO>::field(a.out, a.out_fs, b).at((int64_t)col * a.out_ld);
#pragma unroll
      for (int j = 0; j < G::NIN; ++j) {
        const int d = window_dst(a.rows, G::TIN * j + s);
        if (d >= 0) dst.st(d, v[j]);
      }
    }
  } else if constexpr (MODE == COL_CONV_DLAG) {
    // one column per block (bx); line l0 takes field by * NL + l0.  The
    // lines' products G-hat conj(C-hat) are summed through LDS in line order into the
    // block's partial spectrum part[by]; each field's correlation with the
    // filter goes to out as in COL_CONV.
    const int colb = bx;
    const bool colokb = colb < a.H2;
    const int b = by * NL + l0;
    const bool fok = colokb && b < a.B;
    const int bb = b < a.B ? b : 0;
    using TSI2 = typename ST::in2;
    using TSP = typename ST::part;
    const Spec<TSI2> srcc = Spec<TSI2>::field(a.in2, a.in2_fs, bb).at((int64_t)colb * a.in2_ld);
    const Spec<TSI> srcg = Spec<TSI>::field(a.in, a.in_fs, bb).at((int64_t)colb * a.in_ld);
    TF fv[R3];  // filter values, loaded before the transforms
    {
      const TF* f = reinterpret_cast<const TF*>(a.filt) + (int64_t)(colokb ? colb : 0) * a.filt_ld;
#pragma unroll
      for (int k2 = 0; k2 < R3; ++k2) fv[k2] = (s < G::TOUT && fok) ? f[s + G::TOUT * k2] : (TF)0;
    }
    cx<TC> wc[R3], wg[R3];
    col_fwd<TC, TSI2, R1, R2, R3>(srcc, a.in2_off, a.in2_cnt, fok, s, L, tb, wc);  // C-hat
    col_fwd<TC, TSI, R1, R2, R3>(srcg, a.in_off, a.in_cnt, fok, s, L, tb, wg);    // G-hat
    __syncthreads();
    if (s < G::TOUT) {
#pragma unroll
      for (int k2 = 0; k2 < R3; ++k2) {
        L[s + G::TOUT * k2] = fok ? cmulc(wg[k2], wc[k2]) : mk<TC>(0, 0);
        if (fok) wg[k2] = cscale(wg[k2], fv[k2]);
      }
    }
    __syncthreads();
    if (l0 == 0 && s < G::TOUT && colokb) {
      const cx<TC>* L0 = reinterpret_cast<const cx<TC>*>(smem_raw);
      const Spec<TSP> p = Spec<TSP>::field(a.part, a.part_fs, by).at((int64_t)colb * a.part_ld);
#pragma unroll
      for (int k2 = 0; k2 < R3; ++k2) {
        cx<TC> acc = L0[s + G::TOUT * k2];
        for (int li = 1; li < NL; ++li) acc = acc + L0[(size_t)li * G::EX + s + G::TOUT * k2];
        p.st(s + G::TOUT * k2, acc);
      }
    }
    cx<TC> v[G::NIN];
    xf_inv<TC, R1, R2, R3>(wg, s, L, tb, v);
    if (s < G::TIN && fok) {
      const Spec<TSO> dst = Spec<TSO>::field(a.out, a.out_fs, b).at((int64_t)colb * a.out_ld);
#pragma unroll
      for (int j = 0; j < G::NIN; ++j) {
        const int d = window_dst(a.rows, G::TIN * j + s);
        if (d >= 0) dst.st(d, v[j]);
      }
    }
  } else if constexpr (MODE == COL_FWD_REAL) {
    // forward transform of the input columns; store Re(X) * scale (natural order)
    const int b = by;
    const Spec<TSI> src = Spec<TSI>::field(a.in, a.in_fs, b).at((int64_t)col * a.in_ld);
    cx<TC> w[R3];
    col_fwd<TC, TSI, R1, R2, R3>(src, a.in_off, a.in_cnt, colok, s, L, tb, w);
    if (s < G::TOUT && colok) {
      TSO* dst = reinterpret_cast<TSO*>(a.out) + (int64_t)b * a.out_fs + (int64_t)col * a.out_ld;
#pragma unroll
      for (int k2 = 0; k2 < R3; ++k2) dst[s + G::TOUT * k2] = (TSO)(w[k2].x * (TC)a.scale);
    }
  } else if constexpr (MODE == COL_CE) {
    // sampler pass 1: column k2 (all ncol_full frequencies) of sqrt(Lambda/N) (xi1 + i xi2),
    // xi from Philox counter (k1 * ncol_full + k2, pair, STREAM_CE, 0); forward transform
    // over k1; keep rows [0, rows.na) -> out[pair][k2][r]
    const int pair = a.pair0 + by;
    const int kk2 = col < a.ncol_full - col ? col : a.ncol_full - col;  // Lambda is even
    const double* lam = reinterpret_cast<const double*>(a.filt) + (int64_t)kk2 * a.filt_ld;
    cx<TC> v[G::NIN];
    if (s < G::TIN) {
#pragma unroll
      for (int j = 0; j < G::NIN; ++j) {
        const int k1 = G::TIN * j + s;
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
        v[j] = z;
      }
    }
    cx<TC> w[R3];
    xf_fwd<TC, R1, R2, R3, -1>(v, w, s, L, tb);
    if (s < G::TOUT && colok) {
      const Spec<TSO> dst = Spec<TSO>::field(a.out, a.out_fs, by).at((int64_t)col * a.out_ld);
#pragma unroll
      for (int k2 = 0; k2 < R3; ++k2) {
        const int d = window_dst(a.rows, s + G::TOUT * k2);
        if (d >= 0) dst.st(d, w[k2]);
      }
    }
  } else {  // COL_INV_SUM: inverse transform of sum_g part[g] (natural order), keep rows
    cx<TC> v[G::NIN];
#pragma unroll
    for (int j = 0; j < G::NIN; ++j) v[j] = mk<TC>(0, 0);
    if (s < G::TIN && colok) {
      // four partials per round: their 4 NIN loads go out together; every element is
      // still summed in the order g = 0, 1, ...
      for (int g0 = 0; g0 < a.G; g0 += 4) {
        typename Spec<TSI>::raw t[4][G::NIN];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const Spec<TSI> pg = Spec<TSI>::field(a.in, a.in_fs, g0 + u < a.G ? g0 + u : g0).at((int64_t)col * a.in_ld + s);
#pragma unroll
          for (int j = 0; j < G::NIN; ++j) t[u][j] = pg.ldraw(G::TIN * j);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (g0 + u < a.G) {
#pragma unroll
            for (int j = 0; j < G::NIN; ++j) v[j] = v[j] + Spec<TSI>::template cvt<TC>(t[u][j]);
          }
      }
    }
    cx<TC> w[R3];
    xf_fwd<TC, R1, R2, R3, 1>(v, w, s, L, tb);
    if (s < G::TOUT && colok) {
      const Spec<TSO> dst = Spec<TSO>::field(a.out, 0, 0).at((int64_t)col * a.out_ld);
#pragma unroll
      for (int k2 = 0; k2 < R3; ++k2) {
        const int d = window_dst(a.rows, s + G::TOUT * k2);
        if (d >= 0) dst.st(d, w[k2]);
      }
    }
  }
}

// ----------------------------------------------------------------------------------------
// row kernel: inverse (frequency-major half spectra -> real rows), two rows per line
// ----------------------------------------------------------------------------------------
// Loads the block's rows (transposed through LDS) and forms line l's complex input
// Xa + i Xb from the half spectra (conjugate symmetry for k > F/2).
template <typename TC, int R1, int R2, int R3>
__device__ __forceinline__ void c2r_line_input(const cx<TC>* T, int R2b, int l, int s, int H2,
                                               cx<TC> (&v)[(Geo<R1, R2, R3>::NIN)]) {
  using G = Geo<R1, R2, R3>;
  if (s < G::TIN) {
#pragma unroll
    for (int j = 0; j < G::NIN; ++j) {
      const int k = G::TIN * j + s;
      const bool lo = k < H2;
      const int kk = lo ? k : G::F - k;
      cx<TC> xa = T[tpos(kk, 2 * l, R2b)], xb = T[tpos(kk, 2 * l + 1, R2b)];
      if (kk == 0 || 2 * kk == G::F) { xa.y = 0; xb.y = 0; }  // DC / Nyquist are real
      if (!lo) { xa.y = -xa.y; xb.y = -xb.y; }
      v[j] = mk<TC>(xa.x - xb.y, xa.y + xb.x);  // Xa + i Xb
    }
  }
}

template <typename TC, typename TS, typename TO, int R1, int R2, int R3>
KRIG_ROW_KERNEL k_rows_c2r(RowsC2RArgs a) {
  int bx, by;
  logical_block<false>(bx, by);
  using G = Geo<R1, R2, R3>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<TC>* lds = reinterpret_cast<cx<TC>*>(smem_raw);
  const int s = threadIdx.x % G::NT;
  const int l = threadIdx.x / G::NT;
  const int NL = a.NL;
  const int b = by;
  const int row0 = 2 * bx * NL;
  const int ra = row0 + 2 * l, rb = ra + 1;
  const bool oka = ra < a.nrows, okb = rb < a.nrows;
  const cx<TC>* twF = reinterpret_cast<const cx<TC>*>(a.twF);
  const TwB<TC> tb = tw_bases<TC, R1, R2, R3, false>(twF, s);
  // row-contiguous loads of the block's 2 NL rows into T[k][rl]
  const int R2b = 2 * NL;
  cx<TC>* T = lds;
  const Spec<TS> in = Spec<TS>::field(a.in, a.in_fs, b);
  {
    // a thread's share is at most IT elements (blockDim = NT * NL, H2 = F/2 + 1): all
    // its loads are issued before the first LDS store
    // element idx = k R2b + rl goes to thread idx mod blockDim (NT NL)
    constexpr int IT = (2 * (G::F / 2 + 1) + G::NT - 1) / G::NT;
    typename Spec<TS>::raw buf[IT];
    {
      TWalk<G::NT> e(threadIdx.x, NL);
#pragma unroll
      for (int it = 0; it < IT; ++it, e.next()) {
        const int row = row0 + e.rl;
        buf[it] = (e.k < a.H2 && row < a.nrows) ? in.ldraw((int64_t)e.k * a.in_ld + row) : Spec<TS>::zero();
      }
    }
    TWalk<G::NT> e(threadIdx.x, NL);
#pragma unroll
    for (int it = 0; it < IT; ++it, e.next())
      if (e.k < a.H2) T[tpos(e.k, e.rl, R2b)] = Spec<TS>::template cvt<TC>(buf[it]);
  }
  __syncthreads();
  cx<TC> v[G::NIN];
  c2r_line_input<TC, R1, R2, R3>(T, R2b, l, s, a.H2, v);
  cx<TC>* L = lds + (size_t)l * G::ROWS;
  cx<TC> w[R3];
  xf_fwd<TC, R1, R2, R3, 1>(v, w, s, L, tb);
  if (s < G::TOUT) {
    TO* oa = reinterpret_cast<TO*>(a.out) + (int64_t)b * a.out_fs + (int64_t)ra * a.ldo;
    TO* ob = oa + a.ldo;
    const TO* ad = reinterpret_cast<const TO*>(a.add);
#pragma unroll
    for (int k2 = 0; k2 < R3; ++k2) {
      const int c = s + G::TOUT * k2;
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
template <typename TC, typename TO, int R1, int R2, int R3>
__global__ void __launch_bounds__(256) k_rows_c2r_fold(RowsC2RArgs a) {
  int bx, by;
  logical_block<false>(bx, by);
  using G = Geo<R1, R2, R3>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<TC>* lds = reinterpret_cast<cx<TC>*>(smem_raw);
  const int s = threadIdx.x % G::NT;
  const int l = threadIdx.x / G::NT;
  const int NL = a.NL;
  const int n1l = a.nrows, n2l = a.cols.na;
  const int row0 = 2 * bx * NL;
  const int ra = row0 + 2 * l, rb = ra + 1;
  const cx<TC>* twF = reinterpret_cast<const cx<TC>*>(a.twF);
  const TwB<TC> tb = tw_bases<TC, R1, R2, R3, false>(twF, s);
  const int R2b = 2 * NL;
  cx<TC>* T = lds;
  const cx<TC>* in = reinterpret_cast<const cx<TC>*>(a.in);
  {
    constexpr int IT = (2 * (G::F / 2 + 1) + G::NT - 1) / G::NT;  // as in k_rows_c2r
    cx<TC> b0[IT], b1[IT];
    {
      TWalk<G::NT> e(threadIdx.x, NL);
#pragma unroll
      for (int it = 0; it < IT; ++it, e.next()) {
        const int u = row0 + e.rl;
        const bool ok = e.k < a.H2 && u < n1l;
        b0[it] = ok ? in[(int64_t)e.k * a.in_ld + u] : mk<TC>(0, 0);
        b1[it] = (ok && u > 0) ? in[(int64_t)e.k * a.in_ld + 2 * n1l - 1 - u] : mk<TC>(0, 0);
      }
    }
    TWalk<G::NT> e(threadIdx.x, NL);
#pragma unroll
    for (int it = 0; it < IT; ++it, e.next()) {
      const int u = row0 + e.rl;
      if (e.k < a.H2) T[tpos(e.k, e.rl, R2b)] = u > 0 ? b0[it] + b1[it] : b0[it];
    }
  }
  __syncthreads();
  cx<TC> v[G::NIN];
  c2r_line_input<TC, R1, R2, R3>(T, R2b, l, s, a.H2, v);
  cx<TC>* L = lds + (size_t)l * G::ROWS;
  cx<TC> w[R3];
  xf_fwd<TC, R1, R2, R3, 1>(v, w, s, L, tb);
  __syncthreads();
  if (s < G::TOUT) {
#pragma unroll
    for (int k2 = 0; k2 < R3; ++k2) L[s + G::TOUT * k2] = w[k2];  // natural column order
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
template <typename TC, typename TS, typename TO, int R1, int R2, int R3>
__global__ void __launch_bounds__(256) k_rows_ce(RowsCEArgs a) {
  int bx, by;
  logical_block<false>(bx, by);
  using G = Geo<R1, R2, R3>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<TC>* lds = reinterpret_cast<cx<TC>*>(smem_raw);
  const int s = threadIdx.x % G::NT;
  const int l = threadIdx.x / G::NT;
  const int NL = a.NL;
  const int pair = a.pair0 + by;
  const int row0 = bx * NL;
  const int row = row0 + l;
  const cx<TC>* twF = reinterpret_cast<const cx<TC>*>(a.twF);
  const TwB<TC> tb = tw_bases<TC, R1, R2, R3, false>(twF, s);
  const cx<TS>* in = reinterpret_cast<const cx<TS>*>(a.in) + (int64_t)by * a.in_fs;
  cx<TC>* T = lds;  // [k][l]
  {
    // element idx = k NL + rl goes to thread idx mod blockDim (NT NL): a thread keeps
    // its rl and steps k by NT
    constexpr int IT = (G::F + G::NT - 1) / G::NT;
    const int rl = threadIdx.x % NL, k0 = threadIdx.x / NL;
    const int r = row0 + rl;
    cx<TS> buf[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int k = k0 + it * G::NT;
      buf[it] = (k < G::F && r < a.nrows) ? in[(int64_t)k * a.in_ld + r] : mk<TS>(0, 0);
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int k = k0 + it * G::NT;
      if (k < G::F) T[tpos(k, rl, NL)] = ccast<TC>(buf[it]);
    }
  }
  __syncthreads();
  cx<TC> v[G::NIN];
  if (s < G::TIN) {
#pragma unroll
    for (int j = 0; j < G::NIN; ++j) v[j] = T[tpos(G::TIN * j + s, l, NL)];
  }
  cx<TC>* L = lds + (size_t)l * G::EX;
  cx<TC> w[R3];
  xf_fwd<TC, R1, R2, R3, -1>(v, w, s, L, tb);
  if (s < G::TOUT && row < a.nrows) {
    const int re = 2 * pair, im = 2 * pair + 1;
    TO* o1 = reinterpret_cast<TO*>(a.out) + (int64_t)re * a.out_fs + (int64_t)row * a.ldo;
    TO* o2 = reinterpret_cast<TO*>(a.out) + (int64_t)im * a.out_fs + (int64_t)row * a.ldo;
#pragma unroll
    for (int k2 = 0; k2 < R3; ++k2) {
      const int c = s + G::TOUT * k2;
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
template <typename TC, typename TIN, typename TS, int R1, int R2, int R3, int SRC>
hipError_t launch_rows_r2c(const RowsR2CArgs& a, int B, hipStream_t st) {
  using G = Geo<R1, R2, R3>;
  const int npairs = (a.nrows + 1) / 2;
  dim3 grid((npairs + a.NL - 1) / a.NL, B);
  dim3 block(G::NT * a.NL);
  const size_t sh = rows_lds(G::g, a.NL, sizeof(cx<TC>));
  k_rows_r2c<TC, TIN, TS, R1, R2, R3, SRC><<<grid, block, sh, st>>>(a);
  return hipGetLastError();
}

template <typename TF, typename TI, typename ST, int R1, int R2, int R3, int MODE>
hipError_t launch_cols(const ColsArgs& a, int nblk_y, hipStream_t st) {
  using G = Geo<R1, R2, R3>;
  // the lag-gradient pass: one column per block, its NL lines are fields
  dim3 grid(MODE == COL_CONV_DLAG ? a.H2 : (a.H2 + a.NL - 1) / a.NL, nblk_y);
  dim3 block(G::NT * a.NL);
  const size_t sh = cols_lds(G::g, a.NL, sizeof(cx<TF>));
  k_cols<TF, TI, ST, R1, R2, R3, MODE><<<grid, block, sh, st>>>(a);
  return hipGetLastError();
}

template <typename TC, typename TS, typename TO, int R1, int R2, int R3>
hipError_t launch_rows_c2r(const RowsC2RArgs& a, int B, hipStream_t st) {
  using G = Geo<R1, R2, R3>;
  if (a.H2 != G::F / 2 + 1 || a.NL < 1) return hipErrorInvalidValue;  // the load loop's bound
  const int npairs = (a.nrows + 1) / 2;
  dim3 grid((npairs + a.NL - 1) / a.NL, B);
  dim3 block(G::NT * a.NL);
  const size_t sh = rows_lds(G::g, a.NL, sizeof(cx<TC>));
  k_rows_c2r<TC, TS, TO, R1, R2, R3><<<grid, block, sh, st>>>(a);
  return hipGetLastError();
}

template <typename TC, typename TO, int R1, int R2, int R3>
hipError_t launch_rows_c2r_fold(const RowsC2RArgs& a, int B, hipStream_t st) {
  using G = Geo<R1, R2, R3>;
  if (a.H2 != G::F / 2 + 1 || a.NL < 1) return hipErrorInvalidValue;
  const int npairs = (a.nrows + 1) / 2;
  dim3 grid((npairs + a.NL - 1) / a.NL, 1);
  dim3 block(G::NT * a.NL);
  const size_t sh = rows_lds(G::g, a.NL, sizeof(cx<TC>));
  (void)B;
  k_rows_c2r_fold<TC, TO, R1, R2, R3><<<grid, block, sh, st>>>(a);
  return hipGetLastError();
}

template <typename TC, typename TS, typename TO, int R1, int R2, int R3>
hipError_t launch_rows_ce(const RowsCEArgs& a, int npairs, hipStream_t st) {
  using G = Geo<R1, R2, R3>;
  dim3 grid((a.nrows + a.NL - 1) / a.NL, npairs);
  dim3 block(G::NT * a.NL);
  const size_t sh = ce_rows_lds(G::g, a.NL, sizeof(cx<TC>));
  k_rows_ce<TC, TS, TO, R1, R2, R3><<<grid, block, sh, st>>>(a);
  return hipGetLastError();
}

template <int R1, int R2, int R3>
FftEntry make_fft_entry() {
  FftEntry e;
  e.F = R1 * R2 * R3;
  e.geo = fft_geo(R1, R2, R3);
  FftSet& k = e.k;
  using S64 = Stor<double, double, double, double>;
  using S32 = Stor<float, float, float, float>;
  k.r2c_csr = launch_rows_r2c<double, double, double, R1, R2, R3, SRC_CSR>;
  k.r2c_dense_f64 = launch_rows_r2c<double, double, double, R1, R2, R3, SRC_DENSE>;
  k.r2c_lag = launch_rows_r2c<double, double, double, R1, R2, R3, SRC_LAG>;
  k.conv64 = launch_cols<double, double, S64, R1, R2, R3, COL_CONV>;
  k.conv_dlag64 = launch_cols<double, double, S64, R1, R2, R3, COL_CONV_DLAG>;
  k.fwd_real64 = launch_cols<double, double, S64, R1, R2, R3, COL_FWD_REAL>;
  k.inv_sum64 = launch_cols<double, double, S64, R1, R2, R3, COL_INV_SUM>;
  k.c2r64 = launch_rows_c2r<double, double, double, R1, R2, R3>;
  k.c2r64_32 = launch_rows_c2r<double, double, float, R1, R2, R3>;
  // FP32 plans' adjoint: FP64 arithmetic, FP32 spectra where their rounding stays harmless
  k.r2c_dense_f32 = launch_rows_r2c<double, float, float, R1, R2, R3, SRC_DENSE>;
  k.conv_adj_f = launch_cols<double, double, Stor<float, float, double, float>, R1, R2, R3, COL_CONV>;
  k.conv_dlag_f = launch_cols<double, double, Stor<float, double, double, float>, R1, R2, R3, COL_CONV_DLAG>;
  k.inv_sum_f = launch_cols<double, double, Stor<float, float, double, double>, R1, R2, R3, COL_INV_SUM>;
  k.c2r_fold32 = launch_rows_c2r_fold<double, float, R1, R2, R3>;
  k.c2r_fold64 = launch_rows_c2r_fold<double, double, R1, R2, R3>;
  k.r2c_cov = launch_rows_r2c<double, double, double, R1, R2, R3, SRC_COV>;
  k.r2c_center = launch_rows_r2c<double, double, double, R1, R2, R3, SRC_CENTER>;
  k.r2c_delta = launch_rows_r2c<double, double, double, R1, R2, R3, SRC_DELTA>;
  k.ce_cols32 = launch_cols<float, float, S32, R1, R2, R3, COL_CE>;
  k.ce_cols64 = launch_cols<double, double, S64, R1, R2, R3, COL_CE>;
  k.ce_rows32 = launch_rows_ce<float, float, float, R1, R2, R3>;
  k.ce_rows64 = launch_rows_ce<double, double, double, R1, R2, R3>;
  return e;
}

}  // namespace krig

#define KRIG_FFT_SIZE(R1, R2, R3)                                                               \
  namespace krig {                                                                              \
  void register_fft_##R1##x##R2##x##R3() { register_fft(make_fft_entry<R1, R2, R3>()); }        \
  }
