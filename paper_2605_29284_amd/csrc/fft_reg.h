// Register-resident DFTs of small compile-time lengths (2..64, factors 2 and 3).
//
// DFT<N, DIR, T>::run(v) replaces v[0..N) by its DFT  X[k] = sum_n v[n] exp(DIR 2 pi i nk/N)
// (DIR = -1 forward, +1 inverse, unnormalised), natural order in and out.  The
// recursion is a mixed-radix decimation in time fully unrolled at compile time,
// so every array index is a constant and the data never leave registers; all
// twiddles are compile-time constants computed in double precision.
#pragma once
#include "krig_internal.h"

namespace krig {

__host__ __device__ constexpr int dft_split(int N) {
  // first radix of the decomposition N = R * S
  return (N % 4 == 0 && N > 4) ? 4 : ((N % 2 == 0 && N > 3) ? 2 : 3);
}

template <int N, int DIR, typename T> struct DFT;

template <int DIR, typename T> struct DFT<1, DIR, T> {
  static __host__ __device__ __forceinline__ void run(cx<T>*) {}
};

template <int DIR, typename T> struct DFT<2, DIR, T> {
  static __host__ __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <int DIR, typename T> struct DFT<3, DIR, T> {
  static __host__ __device__ __forceinline__ void run(cx<T>* v) {
    // X1,2 = a - (b+c)/2 -/+ (DIR) i (sqrt3/2)(b-c) ; with w = exp(DIR 2 pi i/3)
    constexpr T h = (T)0.86602540378443864676372317075294;  // sqrt(3)/2
    cx<T> a = v[0], b = v[1], c = v[2];
    cx<T> t1 = b + c;
    cx<T> t2 = mk<T>(a.x - (T)0.5 * t1.x, a.y - (T)0.5 * t1.y);
    cx<T> d = b - c;
    cx<T> t3 = muli<DIR>(mk<T>(h * d.x, h * d.y));
    v[0] = a + t1;
    v[1] = t2 + t3;
    v[2] = t2 - t3;
  }
};

template <int DIR, typename T> struct DFT<4, DIR, T> {
  static __host__ __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> a = v[0], b = v[1], c = v[2], d = v[3];
    cx<T> s0 = a + c, d0 = a - c, s1 = b + d, d1 = muli<DIR>(b - d);
    v[0] = s0 + s1;
    v[2] = s0 - s1;
    v[1] = d0 + d1;
    v[3] = d0 - d1;
  }
};

template <int N, int DIR, typename T> struct DFT {
  static constexpr int R = dft_split(N);
  static constexpr int S = N / R;
  static_assert(R * S == N, "DFT length must have factors 2 and 3 only");
  static __host__ __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> sub[R][S];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int s = 0; s < S; ++s) sub[r][s] = v[R * s + r];
#pragma unroll
    for (int r = 0; r < R; ++r) DFT<S, DIR, T>::run(sub[r]);
    sfor<0, S>([&](auto k2c) {
      constexpr int k2 = decltype(k2c)::value;
      cx<T> t[R];
      sfor<0, R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        t[r] = twmul<r * k2, N, DIR>(sub[r][k2]);
      });
      DFT<R, DIR, T>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < R; ++k1) v[k2 + S * k1] = t[k1];
    });
  }
};

}  // namespace krig
