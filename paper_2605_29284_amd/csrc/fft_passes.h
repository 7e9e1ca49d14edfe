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

// Threads outside a pass's range read entry 0, which is exactly 1 (d = 0).  S > 1 reads
// the powers of W_F from the table of length S F (entry S j = W_(S F)^(S j) = W_F^j).
// t2: the thread's index in the middle pass (t itself, or its remapped index: see xf_fwd).
template <typename TC, int R1, int R2, int R3, bool INV, int S = 1>
__device__ __forceinline__ TwB<TC> tw_bases(const cx<TC>* tw, int t, int t2) {
  using G = Geo<R1, R2, R3>;
  const cx<float>* td = reinterpret_cast<const cx<float>*>(tw + S * G::F);
  const int j1 = S * ((G::THREE && t < G::TIN) ? t : 0);
  const int j2 = S * (t2 < G::T2 ? R1 * (t2 % R3) : 0);
  const int j3 = S * ((INV && t < G::TOUT) ? R1 * (t / R1) : 0);
  const int j4 = S * ((INV && G::THREE && t2 < G::T2) ? R3 * (t2 / R3) : 0);
  TwB<TC> b;
  b.f1 = tw[j1];
  b.f2 = tw[j2];
  b.i3 = tw[j3];
  b.i4a = tw[S * ((INV && G::THREE && t2 < G::T2) ? (t2 / R3) * (t2 % R3) : 0)];
  b.i4b = tw[j4];
  b.d1 = td[j1];
  b.d2 = td[j2];
  b.d3 = td[j3];
  b.d4 = td[j4];
  return b;
}
template <typename TC, int R1, int R2, int R3, bool INV, int S = 1>
__device__ __forceinline__ TwB<TC> tw_bases(const cx<TC>* tw, int t) {
  return tw_bases<TC, R1, R2, R3, INV, S>(tw, t, t);
}

// The middle pass of a three-pass transform runs on T2 of a line's NT threads and only
// exchanges through LDS between block barriers, so any thread of the block may do it for any
// line.  Remapped, block thread T works on line T / T2 as its thread T mod T2: the busy
// threads fill whole waves and the rest (NL (NT - T2) threads, e.g. one wave of three at
// length 768 = 8 x 12 x 8 with two lines) skip the pass instead of issuing it half masked.
// Returns the line for the middle pass (NL or more: none); t2 receives the index.
template <int R1, int R2, int R3>
__device__ __forceinline__ int mid_line(int T, int NL, int& t2) {
  using G = Geo<R1, R2, R3>;
  if constexpr (G::THREE) {
    const int l2 = T / G::T2;
    t2 = l2 < NL ? T % G::T2 : G::T2;
    return l2;
  } else {
    t2 = T % G::NT;  // two-stage forms take their middle input from registers: no remap
    return T / G::NT;
  }
}

// The lines of a block share its barrier (a line may span two waves); a line that is exactly
// one wave (the paired column kernels) needs only its own LDS accesses ordered: a wave's LDS
// operations execute in issue order, and the fences keep the compiler from moving them.
template <bool WAVE>
__device__ __forceinline__ void sync_lines() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
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
// t2, L2: the thread's middle-pass index and the LDS slots of the line it does that pass for
// (mid_line), or t and L.
template <typename TC, int R1, int R2, int R3, int DIR, bool WAVE = false>
__device__ __forceinline__ void xf_fwd(cx<TC> (&v)[(Geo<R1, R2, R3>::NIN)], cx<TC> (&w)[R3], int t, cx<TC>* L,
                                       const TwB<TC>& tb, int t2, cx<TC>* L2) {
  using G = Geo<R1, R2, R3>;
  sync_lines<WAVE>();
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
    sync_lines<WAVE>();
    if (t2 < G::T2) {
      const int k1 = t2 / R3, s = t2 % R3;
#pragma unroll
      for (int n1 = 0; n1 < R2; ++n1) u[n1] = L2[k1 * G::P1 + R3 * n1 + s];
    }
    sync_lines<WAVE>();
  } else {
#pragma unroll
    for (int n1 = 0; n1 < R2; ++n1) u[n1] = v[n1];
  }
  if (t2 < G::T2) {
    const int k1 = t2 / R3, s = t2 % R3;
    DFT<R2, DIR, TC>::run(u);
    cx<TC>* Lk = L2 + k1 * G::RS;
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
  sync_lines<WAVE>();
  if (t < G::TOUT) {
    const int k1 = t % R1, sp = t / R1;
    const cx<TC>* Lk = L + k1 * G::RS;
#pragma unroll
    for (int n2 = 0; n2 < R3; ++n2) w[n2] = Lk[n2 * G::ON2 + sp];
    DFT<R3, DIR, TC>::run(w);
  }
}

template <typename TC, int R1, int R2, int R3, int DIR, bool WAVE = false>
__device__ __forceinline__ void xf_fwd(cx<TC> (&v)[(Geo<R1, R2, R3>::NIN)], cx<TC> (&w)[R3], int t, cx<TC>* L,
                                       const TwB<TC>& tb) {
  xf_fwd<TC, R1, R2, R3, DIR, WAVE>(v, w, t, L, tb, t, L);
}

// Inverse transform from the output layout (thread t < TOUT holds X[t + TOUT k2])
// back to the input layout (thread t < TIN ends with x[t + TIN j] in v[j]): the
// passes of xf_fwd in reverse with conjugate twiddles.
template <typename TC, int R1, int R2, int R3, bool WAVE = false>
__device__ __forceinline__ void xf_inv(cx<TC> (&w)[R3], int t, cx<TC>* L, const TwB<TC>& tb,
                                       cx<TC> (&v)[(Geo<R1, R2, R3>::NIN)], int t2, cx<TC>* L2) {
  using G = Geo<R1, R2, R3>;
  sync_lines<WAVE>();
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
  sync_lines<WAVE>();
  cx<TC> u[R2];
  // the middle pass reads (and, three-pass, writes) the remapped line; a two-stage form
  // keeps its values in the thread's own registers (t2 = t there)
  if (t2 < G::T2) {
    const int k1 = t2 / R3, n2 = t2 % R3;
#pragma unroll
    for (int q = 0; q < R2; ++q) u[q] = L2[k1 * G::RS + n2 * G::ON2 + q];
  }
  if constexpr (G::THREE) {
    sync_lines<WAVE>();
    if (t2 < G::T2) {
      const int k1 = t2 / R3, n2 = t2 % R3;
      DFT<R2, 1, TC>::run(u);
      cx<TC> wm = tb.i4a;  // W^(m k1), m = R3 n1 + n2
#pragma unroll
      for (int n1 = 0; n1 < R2; ++n1) {
        const int m = R3 * n1 + n2;
        if (n1 > 0) wm = cmul(wm, tb.i4b);
        if (n1 > 0 && n1 % 4 == 0) wm = tw_fix(wm, tb.d4, 4);
        L2[k1 * G::P1 + m] = cmulc(u[n1], wm);
      }
    }
    sync_lines<WAVE>();
    if (t < G::TIN) {
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) v[k1] = L[k1 * G::P1 + t];
      DFT<R1, 1, TC>::run(v);
    }
  } else {
    if (t2 < G::T2) {
      DFT<R2, 1, TC>::run(u);
#pragma unroll
      for (int n1 = 0; n1 < R2; ++n1) v[n1] = u[n1];
    }
  }
}

template <typename TC, int R1, int R2, int R3, bool WAVE = false>
__device__ __forceinline__ void xf_inv(cx<TC> (&w)[R3], int t, cx<TC>* L, const TwB<TC>& tb,
                                       cx<TC> (&v)[(Geo<R1, R2, R3>::NIN)]) {
  xf_inv<TC, R1, R2, R3, WAVE>(w, t, L, tb, v, t, L);
}

// ----------------------------------------------------------------------------------------
// row kernels: forward (real rows -> frequency-major half spectra)
// ----------------------------------------------------------------------------------------
enum { SRC_CSR = 0, SRC_DENSE = 1, SRC_LAG = 2, SRC_COV = 3, SRC_CENTER = 4, SRC_DELTA = 5, SRC_CSR_SCALED = 6 };

// Kernel bodies (fft_body_*.inc) are included inside the kernels, after the block's logical
// coordinates (bx: row or column block, by: field or group) are set, so that one text serves a
// plain launch (one problem, block id -> (bx, by)) and the persistent launch of an uneven batch
// (a tile list over several problems).  Included rather than called: the call form changed the
// register allocation of the plain kernels (two of them spilled).

template <typename TC, typename TIN, typename TS, int R1, int R2, int R3, int SRC>
KRIG_ROW_KERNEL k_rows_r2c(RowsR2CArgs a) {
  int bx, by;
  logical_block<false>(bx, by);
#include "fft_body_rows_r2c.inc"
}

// ----------------------------------------------------------------------------------------
// column kernels (contiguous columns of frequency-major spectra)
// ----------------------------------------------------------------------------------------
template <typename TC, typename TS, int R1, int R2, int R3>
__device__ __forceinline__ void col_fwd(const Spec<TS> src, int in_off, int in_cnt, bool colok, int s,
                                        cx<TC>* L, const TwB<TC>& tb, cx<TC> (&w)[R3], int t2, cx<TC>* L2) {
  using G = Geo<R1, R2, R3>;
  cx<TC> v[G::NIN];
  if (s < G::TIN) {
#pragma unroll
    for (int j = 0; j < G::NIN; ++j) {
      const int r = G::TIN * j + s - in_off;
      v[j] = (colok && r >= 0 && r < in_cnt) ? src.template ld<TC>(r) : mk<TC>(0, 0);
    }
  }
  xf_fwd<TC, R1, R2, R3, -1>(v, w, s, L, tb, t2, L2);
}

enum { COL_CONV = 0, COL_CONV_DLAG = 1, COL_FWD_REAL = 2, COL_INV_SUM = 3, COL_CE = 4 };

// The lag-gradient column pass (two forward transforms and an inverse per line) of the
// same forms needs 160 VGPRs: three waves per SIMD without scratch (it loads its filter values
// and inverse twiddle bases late for that), faster than uncapped at two waves; a four-wave cap
// (over 200 bytes of scratch) runs at half speed.  The plain convolution pass keeps the
// default (four waves): a five-wave cap made it spill and run slower.
template <int R1, int R2, int R3, int MODE> struct ColCap {
  static constexpr int waves = (MODE == COL_CONV_DLAG && RowCap<R1, R2, R3>::waves > 1) ? 3 : 1;
};


template <typename TF, typename TI, typename ST, int R1, int R2, int R3, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ColCap<R1, R2, R3, MODE>::waves)))
k_cols(ColsArgs a) {
  int bx, by;
  logical_block<true>(bx, by);
#include "fft_body_cols.inc"
}

// Paired column kernel: columns of length 2 F (F = R1 R2 R3 on at most 64 threads), one wave
// per column, two half-length transforms and a radix-2 butterfly, no block barriers
// (fft_body_cols_pair.inc).  The convolution form only.
template <typename TF, typename TI, typename ST, int R1, int R2, int R3>
__global__ void __launch_bounds__(256) k_cols_pair(ColsArgs a) {
  int bx, by;
  logical_block<true>(bx, by);
#include "fft_body_cols_pair.inc"
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
#include "fft_body_rows_c2r.inc"
}

// Inverse rows of a weighted mixture (MixRowsArgs): per component the rows of
// k_rows_c2r, then lam_k times the kept values added in FP64 in component order; one rounding
// to TO at the end.  The component's spectra pointer is selected with constant indices (no
// dynamic indexing of the argument block).
__device__ __forceinline__ const void* mix_in(const MixRowsArgs& m, int k) {
  switch (k) {
    case 0: return m.in[0];
    case 1: return m.in[1];
    case 2: return m.in[2];
    case 3: return m.in[3];
    case 4: return m.in[4];
    case 5: return m.in[5];
    case 6: return m.in[6];
    default: return m.in[7];
  }
}

// A loop over components lets the compiler hoist everything that depends only on the thread's
// coordinates (twiddle bases and powers, LDS and load addresses) out of it and hold it all in
// registers (about 250 VGPRs); the coordinates and the twiddle pointer are therefore passed
// through an empty asm per component, which makes them opaque, and each component recomputes
// its addresses (133 VGPRs, three waves per SIMD, no scratch; no wave cap).
template <typename TC, typename TS, typename TO, int R1, int R2, int R3>
__global__ void __launch_bounds__(256) k_rows_c2r_mix(MixRowsArgs m) {
  using G = Geo<R1, R2, R3>;
  const RowsC2RArgs& a = m.r;
  int bx, by;
  logical_block<false>(bx, by);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<TC>* lds = reinterpret_cast<cx<TC>*>(smem_raw);
  const int tid0 = threadIdx.x;
  const int NL = a.NL;
  const int b = by;
  const int row0 = 2 * bx * NL;
  const int R2b = 2 * NL;
  cx<TC>* T = lds;
  double acc_a[R3], acc_b[R3];
#pragma unroll
  for (int k2 = 0; k2 < R3; ++k2) acc_a[k2] = acc_b[k2] = 0.0;
#pragma unroll 1
  for (int k = 0; k < m.C; ++k) {
    if (k > 0) __syncthreads();  // every line is done with the previous component's LDS
    const Spec<TS> in = Spec<TS>::field(mix_in(m, k), a.in_fs, b);
    const cx<TC>* twF = reinterpret_cast<const cx<TC>*>(a.twF);
    int tid = tid0;
    asm volatile("" : "+s"(twF), "+v"(tid));
    const int s = tid % G::NT, l = tid / G::NT;
    const int ra = row0 + 2 * l, rb = ra + 1;
    const bool oka = ra < a.nrows, okb = rb < a.nrows;
    cx<TC>* L = lds + (size_t)l * G::ROWS;
    const TwB<TC> tb = tw_bases<TC, R1, R2, R3, false>(twF, s);
    {
      constexpr int IT = (2 * (G::F / 2 + 1) + G::NT - 1) / G::NT;  // as in k_rows_c2r
      typename Spec<TS>::raw buf[IT];
      {
        TWalk<G::NT> e(tid, NL);
#pragma unroll
        for (int it = 0; it < IT; ++it, e.next()) {
          const int row = row0 + e.rl;
          buf[it] = (e.k < a.H2 && row < a.nrows) ? in.ldraw((int64_t)e.k * a.in_ld + row) : Spec<TS>::zero();
        }
      }
      TWalk<G::NT> e(tid, NL);
#pragma unroll
      for (int it = 0; it < IT; ++it, e.next())
        if (e.k < a.H2) T[tpos(e.k, e.rl, R2b)] = Spec<TS>::template cvt<TC>(buf[it]);
    }
    __syncthreads();
    cx<TC> v[G::NIN];
    c2r_line_input<TC, R1, R2, R3>(T, R2b, l, s, a.H2, v);
    cx<TC> w[R3];
    xf_fwd<TC, R1, R2, R3, 1>(v, w, s, L, tb);
    if (s < G::TOUT) {
      const double* lk = m.lam + (int64_t)k * m.lam_cs;
#pragma unroll
      for (int k2 = 0; k2 < R3; ++k2) {
        const int d = window_dst(a.cols, s + G::TOUT * k2);
        if (d >= 0) {
          if (oka) acc_a[k2] += lk[(int64_t)ra * m.lam_ld + d] * (double)w[k2].x;
          if (okb) acc_b[k2] += lk[(int64_t)rb * m.lam_ld + d] * (double)w[k2].y;
        }
      }
    }
  }
  const int s = tid0 % G::NT, l = tid0 / G::NT;
  const int ra = row0 + 2 * l, rb = ra + 1;
  const bool oka = ra < a.nrows, okb = rb < a.nrows;
  if (s < G::TOUT) {
    TO* oa = reinterpret_cast<TO*>(a.out) + (int64_t)b * a.out_fs + (int64_t)ra * a.ldo;
    TO* ob = oa + a.ldo;
#pragma unroll
    for (int k2 = 0; k2 < R3; ++k2) {
      const int d = window_dst(a.cols, s + G::TOUT * k2);
      if (d >= 0) {
        if (oka) oa[d] = (TO)acc_a[k2];
        if (okb) ob[d] = (TO)acc_b[k2];
      }
    }
  }
}

// ----------------------------------------------------------------------------------------
// Persistent launches of an uneven batch: the tiles (row or column blocks) of several
// problems of the same transform form in one list, problem i owning tiles [first[i],
// first[i + 1]) laid out as (bx, by) = (t mod nbx[i], t / nbx[i]) with t the tile's index
// within the problem.  A grid of about one resident round of blocks walks the list, block b
// taking tiles b, b + grid, b + 2 grid, ... until it is exhausted: no block waits for
// another, so every block ends.  (An atomic counter handing out tiles measured twice as slow
// on the batch's ~10^6 small triangular-product tiles.)  Each tile's arithmetic is that of
// the problem's own launch, so results are bitwise the same.
// ----------------------------------------------------------------------------------------
// Argument blocks are read through the constant address space: they do not change while the
// kernel runs, so the compiler may reload a field where it is used instead of holding every
// field in registers across the tile.
template <typename T> using const_as = const __attribute__((address_space(4))) T;

template <typename ArgsT>
__device__ __forceinline__ bool next_tile(const QueueArgs& q, int& iter, int& prob, int& bx, int& by,
                                          const_as<ArgsT>*& a) {
  // the tile index only grows, so the problem is found by stepping forward from the last one
  const int t = blockIdx.x + (iter++) * gridDim.x;
  if (t >= q.total) return false;
  int lo = prob;
  while (lo + 1 < q.count && q.first[lo + 1] <= t) ++lo;
  const int local = t - q.first[lo];
  prob = lo;
  bx = local % q.nbx[lo];
  by = local / q.nbx[lo];
  a = (const_as<ArgsT>*)(q.args) + lo;
  return true;
}

// The queue loop holds a few more registers than a plain launch: the row forms capped at five
// waves per SIMD there run at four here (no scratch).
template <int R1, int R2, int R3> struct QueueRowCap {
  static constexpr int waves = RowCap<R1, R2, R3>::waves > 1 ? 4 : 1;
};
#define KRIG_QUEUE_ROW_KERNEL \
  __global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QueueRowCap<R1, R2, R3>::waves)))

template <typename TC, typename TIN, typename TS, int R1, int R2, int R3, int SRC>
KRIG_QUEUE_ROW_KERNEL k_rows_r2c_queue(QueueArgs q) {
  int prob = 0, bx, by, iter = 0;
  const_as<RowsR2CArgs>* ap;
  while (next_tile(q, iter, prob, bx, by, ap)) {
    const RowsR2CArgs& a = *(const RowsR2CArgs*)ap;
#include "fft_body_rows_r2c.inc"
  }
}

template <typename TF, typename TI, typename ST, int R1, int R2, int R3, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ColCap<R1, R2, R3, MODE>::waves)))
k_cols_queue(QueueArgs q) {
  int prob = 0, bx, by, iter = 0;
  const_as<ColsArgs>* ap;
  while (next_tile(q, iter, prob, bx, by, ap)) {
    const ColsArgs& a = *(const ColsArgs*)ap;
#include "fft_body_cols.inc"
  }
}

template <typename TF, typename TI, typename ST, int R1, int R2, int R3>
__global__ void __launch_bounds__(256) k_cols_pair_queue(QueueArgs q) {
  int prob = 0, bx, by, iter = 0;
  const_as<ColsArgs>* ap;
  while (next_tile(q, iter, prob, bx, by, ap)) {
    const ColsArgs& a = *(const ColsArgs*)ap;
#include "fft_body_cols_pair.inc"
  }
}

template <typename TC, typename TS, typename TO, int R1, int R2, int R3>
KRIG_QUEUE_ROW_KERNEL k_rows_c2r_queue(QueueArgs q) {
  int prob = 0, bx, by, iter = 0;
  const_as<RowsC2RArgs>* ap;
  while (next_tile(q, iter, prob, bx, by, ap)) {
    const RowsC2RArgs& a = *(const RowsC2RArgs*)ap;
#include "fft_body_rows_c2r.inc"
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

// paired columns: NL columns (waves) per block, NL <= 4
template <typename TF, typename TI, typename ST, int R1, int R2, int R3>
hipError_t launch_cols_pair(const ColsArgs& a, int nblk_y, hipStream_t st) {
  using G = Geo<R1, R2, R3>;
  if (a.NL < 1 || a.NL > 4) return hipErrorInvalidValue;
  dim3 grid((a.H2 + a.NL - 1) / a.NL, nblk_y);
  const size_t sh = (size_t)a.NL * G::EX * sizeof(cx<TF>);
  k_cols_pair<TF, TI, ST, R1, R2, R3><<<grid, dim3(64 * a.NL), sh, st>>>(a);
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

template <typename TC, typename TS, typename TO, int R1, int R2, int R3>
hipError_t launch_rows_c2r_mix(const MixRowsArgs& m, int B, hipStream_t st) {
  using G = Geo<R1, R2, R3>;
  const RowsC2RArgs& a = m.r;
  if (a.H2 != G::F / 2 + 1 || a.NL < 1 || m.C < 1 || m.C > MIX_COMP_MAX) return hipErrorInvalidValue;
  const int npairs = (a.nrows + 1) / 2;
  dim3 grid((npairs + a.NL - 1) / a.NL, B);
  dim3 block(G::NT * a.NL);
  const size_t sh = rows_lds(G::g, a.NL, sizeof(cx<TC>));
  k_rows_c2r_mix<TC, TS, TO, R1, R2, R3><<<grid, block, sh, st>>>(m);
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

// a queue launch's grid for nblocks <= 0: one resident round of blocks (occupancy per compute
// unit x compute units) for 0, a d-th of it for -d
template <typename K>
int queue_grid(int nblocks, K kernel, int threads, size_t lds) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, lds) != hipSuccess || per < 1) per = 1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess || cus < 1)
    cus = 1;
  const int round = per * cus;
  return nblocks == 0 ? round : (round / -nblocks > 1 ? round / -nblocks : 1);
}

template <typename TC, typename TIN, typename TS, int R1, int R2, int R3, int SRC>
hipError_t launch_rows_r2c_queue(const QueueArgs& q, int NL, int nblocks, hipStream_t st) {
  using G = Geo<R1, R2, R3>;
  const int threads = G::NT * NL;
  const size_t sh = rows_lds(G::g, NL, sizeof(cx<TC>));
  if (nblocks <= 0) nblocks = queue_grid(nblocks, k_rows_r2c_queue<TC, TIN, TS, R1, R2, R3, SRC>, threads, sh);
  k_rows_r2c_queue<TC, TIN, TS, R1, R2, R3, SRC><<<nblocks, threads, sh, st>>>(q);
  return hipGetLastError();
}

template <typename TF, typename TI, typename ST, int R1, int R2, int R3, int MODE>
hipError_t launch_cols_queue(const QueueArgs& q, int NL, int nblocks, hipStream_t st) {
  using G = Geo<R1, R2, R3>;
  const int threads = G::NT * NL;
  const size_t sh = cols_lds(G::g, NL, sizeof(cx<TF>));
  if (nblocks <= 0) nblocks = queue_grid(nblocks, k_cols_queue<TF, TI, ST, R1, R2, R3, MODE>, threads, sh);
  k_cols_queue<TF, TI, ST, R1, R2, R3, MODE><<<nblocks, threads, sh, st>>>(q);
  return hipGetLastError();
}

template <typename TF, typename TI, typename ST, int R1, int R2, int R3>
hipError_t launch_cols_pair_queue(const QueueArgs& q, int NL, int nblocks, hipStream_t st) {
  using G = Geo<R1, R2, R3>;
  if (NL < 1 || NL > 4) return hipErrorInvalidValue;
  const int threads = 64 * NL;
  const size_t sh = (size_t)NL * G::EX * sizeof(cx<TF>);
  if (nblocks <= 0) nblocks = queue_grid(nblocks, k_cols_pair_queue<TF, TI, ST, R1, R2, R3>, threads, sh);
  k_cols_pair_queue<TF, TI, ST, R1, R2, R3><<<nblocks, threads, sh, st>>>(q);
  return hipGetLastError();
}

template <typename TC, typename TS, typename TO, int R1, int R2, int R3>
hipError_t launch_rows_c2r_queue(const QueueArgs& q, int NL, int nblocks, hipStream_t st) {
  using G = Geo<R1, R2, R3>;
  const int threads = G::NT * NL;
  const size_t sh = rows_lds(G::g, NL, sizeof(cx<TC>));
  if (nblocks <= 0) nblocks = queue_grid(nblocks, k_rows_c2r_queue<TC, TS, TO, R1, R2, R3>, threads, sh);
  k_rows_c2r_queue<TC, TS, TO, R1, R2, R3><<<nblocks, threads, sh, st>>>(q);
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
  k.r2c_csr_scaled = launch_rows_r2c<double, double, double, R1, R2, R3, SRC_CSR_SCALED>;
  k.r2c_dense_f64 = launch_rows_r2c<double, double, double, R1, R2, R3, SRC_DENSE>;
  k.r2c_lag = launch_rows_r2c<double, double, double, R1, R2, R3, SRC_LAG>;
  k.conv64 = launch_cols<double, double, S64, R1, R2, R3, COL_CONV>;
  k.conv_dlag64 = launch_cols<double, double, S64, R1, R2, R3, COL_CONV_DLAG>;
  k.fwd_real64 = launch_cols<double, double, S64, R1, R2, R3, COL_FWD_REAL>;
  k.inv_sum64 = launch_cols<double, double, S64, R1, R2, R3, COL_INV_SUM>;
  k.c2r64 = launch_rows_c2r<double, double, double, R1, R2, R3>;
  // FP32 plans' prediction: the column pass stores its output spectra in FP32
  k.conv_pred_f = launch_cols<double, double, Stor<double, double, float, double>, R1, R2, R3, COL_CONV>;
  k.c2r_f32 = launch_rows_c2r<double, float, float, R1, R2, R3>;
  k.c2r_mix64 = launch_rows_c2r_mix<double, double, double, R1, R2, R3>;
  k.c2r_mix_f32 = launch_rows_c2r_mix<double, float, float, R1, R2, R3>;
  // FP32 plans' adjoint: the FP32 upstream gradient into FP64 spectra
  k.r2c_dense_f32 = launch_rows_r2c<double, float, double, R1, R2, R3, SRC_DENSE>;
  k.c2r_fold32 = launch_rows_c2r_fold<double, float, R1, R2, R3>;
  k.c2r_fold64 = launch_rows_c2r_fold<double, double, R1, R2, R3>;
  k.r2c_cov = launch_rows_r2c<double, double, double, R1, R2, R3, SRC_COV>;
  k.r2c_center = launch_rows_r2c<double, double, double, R1, R2, R3, SRC_CENTER>;
  k.q_r2c_csr = launch_rows_r2c_queue<double, double, double, R1, R2, R3, SRC_CSR>;
  k.q_r2c_dense = launch_rows_r2c_queue<double, double, double, R1, R2, R3, SRC_DENSE>;
  k.q_conv64 = launch_cols_queue<double, double, S64, R1, R2, R3, COL_CONV>;
  k.q_c2r64 = launch_rows_c2r_queue<double, double, double, R1, R2, R3>;
  k.q_conv_pred_f = launch_cols_queue<double, double, Stor<double, double, float, double>, R1, R2, R3, COL_CONV>;
  k.q_c2r_f32 = launch_rows_c2r_queue<double, float, float, R1, R2, R3>;
  k.r2c_delta = launch_rows_r2c<double, double, double, R1, R2, R3, SRC_DELTA>;
  k.ce_cols32 = launch_cols<float, float, S32, R1, R2, R3, COL_CE>;
  k.ce_cols64 = launch_cols<double, double, S64, R1, R2, R3, COL_CE>;
  k.ce_rows32 = launch_rows_ce<float, float, float, R1, R2, R3>;
  k.ce_rows64 = launch_rows_ce<double, double, double, R1, R2, R3>;
  // columns of twice this length, one wave per column (three-pass lengths on exactly 64 threads)
  if constexpr (Geo<R1, R2, R3>::THREE && Geo<R1, R2, R3>::NT == 64) {
    using S64P = Stor<double, double, double, double>;
    using S32P = Stor<double, double, float, double>;
    k.pair_conv64 = launch_cols_pair<double, double, S64P, R1, R2, R3>;
    k.pair_conv_pred_f = launch_cols_pair<double, double, S32P, R1, R2, R3>;
    k.q_pair_conv64 = launch_cols_pair_queue<double, double, S64P, R1, R2, R3>;
    k.q_pair_conv_pred_f = launch_cols_pair_queue<double, double, S32P, R1, R2, R3>;
    k.pair_ex = Geo<R1, R2, R3>::EX;
  }
  return e;
}

}  // namespace krig

#define KRIG_FFT_SIZE(R1, R2, R3)                                                               \
  namespace krig {                                                                              \
  void register_fft_##R1##x##R2##x##R3() { register_fft(make_fft_entry<R1, R2, R3>()); }        \
  }
