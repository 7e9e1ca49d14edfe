// Internal declarations shared by the HIP sources of libkrig (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include <utility>

namespace krig {

// ---------------------------------------------------------------- complex numbers
// Aligned to its full size so that a complex value moves as one 16-byte (FP64) or 8-byte
// (FP32) access: split into two halves, a wave's LDS accesses at a 16-byte stride
// conflict in every bank pair.
template <typename T> struct alignas(2 * sizeof(T)) cx { T x, y; };

template <typename T> __host__ __device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T> __host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T> __host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T> __host__ __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
template <typename T> __host__ __device__ __forceinline__ cx<T> conjg(cx<T> a) { return mk<T>(a.x, -a.y); }
// a * (S i) for S = +1 or -1
template <int S, typename T> __host__ __device__ __forceinline__ cx<T> muli(cx<T> a) {
  return S > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}
template <typename TO, typename TI> __host__ __device__ __forceinline__ cx<TO> ccast(cx<TI> a) {
  return mk<TO>((TO)a.x, (TO)a.y);
}

// ---------------------------------------------------------------- compile-time trigonometry
// cos and sin of 2*pi*J/N for integers J, N, evaluated by the compiler: the angle
// is reduced exactly (integer arithmetic) to the first octant, then a Taylor
// series in double precision (|x| <= pi/4, 14 terms: truncation far below 1 ulp).
constexpr double kPi = 3.14159265358979323846264338327950288;

__host__ __device__ constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
__host__ __device__ constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// returns cos (C=true) or sin (C=false) of 2 pi J / N
__host__ __device__ constexpr double trig_frac(long J, long N, bool want_cos) {
  long r = ((J % N) + N) % N;        // angle = 2 pi r / N in [0, 2 pi)
  long o = (8 * r) / N;              // octant 0..7
  long num = 8 * r - o * N;          // remainder in [0, N): angle = (o + num/N) * pi/4
  double x = (kPi / 4.0) * ((double)num / (double)N);
  double s = taylor_sin(x), c = taylor_cos(x);
  double y = (kPi / 4.0) - x;        // used in odd octants: reflect about pi/4
  double s2 = taylor_sin(y), c2 = taylor_cos(y);
  // (cos, sin) of o*pi/4 + x
  double rc = 0, rs = 0;
  switch (o) {
    case 0: rc = c; rs = s; break;              // [0, pi/4)
    case 1: rc = s2; rs = c2; break;            // pi/2 - y
    case 2: rc = -s; rs = c; break;             // pi/2 + x
    case 3: rc = -c2; rs = s2; break;           // pi - y
    case 4: rc = -c; rs = -s; break;            // pi + x
    case 5: rc = -s2; rs = -c2; break;          // 3pi/2 - y
    case 6: rc = s; rs = -c; break;             // 3pi/2 + x
    default: rc = c2; rs = -s2; break;          // 2pi - y
  }
  return want_cos ? rc : rs;
}

// compile-time loop: f(std::integral_constant<int, I>{}) for I in [B, E)
template <int B, int E, typename F>
__host__ __device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

// a * exp(DIR * 2 pi i J / N), J and N compile-time
template <int J, int N, int DIR, typename T>
__host__ __device__ __forceinline__ cx<T> twmul(cx<T> a) {
  constexpr int r = ((J % N) + N) % N;
  if constexpr (r == 0) {
    return a;
  } else if constexpr (2 * r == N) {
    return mk<T>(-a.x, -a.y);
  } else if constexpr (4 * r == N) {
    return muli<DIR>(a);
  } else if constexpr (4 * r == 3 * N) {
    return muli<-DIR>(a);
  } else {
    constexpr double c = trig_frac(r, N, true);
    constexpr double s = DIR * trig_frac(r, N, false);
    return cmul(a, mk<T>((T)c, (T)s));
  }
}

}  // namespace krig
