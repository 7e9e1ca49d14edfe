// Off-grid predictions from the mesh prediction (the closing discussion of the paper
// suggests predicting on a fine mesh and reaching irregular locations by fast local
// polynomial interpolation): at each point, the tensor-product Lagrange polynomial of
// degree q-1 in x and in y through the q x q mesh nodes around it.
#include "interp.h"

#include <math.h>

namespace krig {

// Lagrange basis on the nodes 0..Q-1 at r in [0, Q-1]: l_a(r) = prod_{k != a} (r - k) / D_a,
// D_a = prod_{k != a} (a - k), an integer.  The numerators come from prefix and suffix
// products; at a node every product is an exact small integer, so l_a is exactly 0 or 1.
template <int Q>
__device__ __forceinline__ void lagrange_basis(double r, double (&l)[Q]) {
  double pre[Q], suf[Q];
  pre[0] = 1.0;
#pragma unroll
  for (int k = 1; k < Q; ++k) pre[k] = pre[k - 1] * (r - (double)(k - 1));
  suf[Q - 1] = 1.0;
#pragma unroll
  for (int k = Q - 2; k >= 0; --k) suf[k] = suf[k + 1] * (r - (double)(k + 1));
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    double d = 1.0;
#pragma unroll
    for (int k = 0; k < Q; ++k)
      if (k != a) d *= (double)(a - k);  // folded at compile time
    l[a] = (pre[a] * suf[a]) / d;
  }
}

// First node of the Q-node stencil around grid coordinate t in [0, m-1]: centred on the
// cell floor(t) (for even Q), shifted inward at the edges.
template <int Q>
__device__ __forceinline__ int stencil_first(double t, int m) {
  const int i0 = (int)floor(t);
  return min(max(i0 + 1 - (Q + 1) / 2, 0), m - Q);
}

// One thread per (point, field): grid (ceil(npts / 256), B).
template <typename TS, int Q>
__global__ void __launch_bounds__(256) k_interp(InterpArgs a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (j >= a.npts) return;
  TS* o = reinterpret_cast<TS*>(a.out) + (int64_t)b * a.out_fs + j;
  const double x = a.pts[2 * (int64_t)j], y = a.pts[2 * (int64_t)j + 1];
  const double t = (x - a.x0) / a.dx, u = (y - a.y0) / a.dy;
  if (!(t >= 0.0 && t <= (double)(a.m1 - 1) && u >= 0.0 && u <= (double)(a.m2 - 1))) {
    *o = (TS)NAN;  // outside the grid's bounding box (also a NaN coordinate)
    return;
  }
  const int sx = stencil_first<Q>(t, a.m1), sy = stencil_first<Q>(u, a.m2);
  double wx[Q], wy[Q];
  lagrange_basis<Q>(t - (double)sx, wx);
  lagrange_basis<Q>(u - (double)sy, wy);
  const TS* base = reinterpret_cast<const TS*>(a.yhat) + (int64_t)b * a.yhat_fs + (int64_t)sx * a.m2 + sy;
  TS v[Q][Q];
#pragma unroll
  for (int p = 0; p < Q; ++p)
#pragma unroll
    for (int c = 0; c < Q; ++c) v[p][c] = base[(int64_t)p * a.m2 + c];
  double acc = 0.0;
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    double row = 0.0;
#pragma unroll
    for (int c = 0; c < Q; ++c) row += wy[c] * (double)v[p][c];
    acc += wx[p] * row;
  }
  *o = (TS)acc;
}

template <typename TS>
hipError_t launch_interp(const InterpArgs& a, int B, int q, hipStream_t st) {
  dim3 grid((a.npts + 255) / 256, B);
  switch (q) {
    case 2: k_interp<TS, 2><<<grid, 256, 0, st>>>(a); break;
    case 3: k_interp<TS, 3><<<grid, 256, 0, st>>>(a); break;
    case 4: k_interp<TS, 4><<<grid, 256, 0, st>>>(a); break;
    case 5: k_interp<TS, 5><<<grid, 256, 0, st>>>(a); break;
    case 6: k_interp<TS, 6><<<grid, 256, 0, st>>>(a); break;
    case 7: k_interp<TS, 7><<<grid, 256, 0, st>>>(a); break;
    case 8: k_interp<TS, 8><<<grid, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t interp_points(const InterpArgs& a, int B, int q, bool f32, hipStream_t st) {
  if (a.npts <= 0 || B <= 0) return hipSuccess;
  if (q < 2 || q > 8 || q > a.m1 || q > a.m2 || B > 65535) return hipErrorInvalidValue;
  return f32 ? launch_interp<float>(a, B, q, st) : launch_interp<double>(a, B, q, st);
}

}  // namespace krig
