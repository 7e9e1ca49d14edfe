// Set-up kernels (Steps 1-4 and the structure of Step 5), the deterministic scatter
// (Steps 5-6, unfused form), the site gather of the adjoint and of conditional
// simulation.
#include "setup.h"

#include "philox_dev.h"

namespace krig {

static inline unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// ------------------------------------------------------------------------------ lag image
__global__ void k_lag_image(GridDev g, MaternDev mt, double* lag64) {
  const int n1l = g.m1 + g.L, n2l = g.m2 + g.L;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n1l * n2l) return;
  const int a = idx / n2l, b = idx % n2l;
  const double hx = a * g.dx, hy = b * g.dy;
  lag64[idx] = matern_cov(sqrt(hx * hx + hy * hy), mt);
}

hipError_t lag_image(const GridDev& g, const MaternDev& mt, double* lag64, hipStream_t st) {
  const int cnt = (g.m1 + g.L) * (g.m2 + g.L);
  hipLaunchKernelGGL(k_lag_image, dim3(nblk(cnt)), dim3(256), 0, st, g, mt, lag64);
  return hipGetLastError();
}

template <typename TO>
__global__ void k_convert(const double* __restrict__ s, TO* __restrict__ d, int64_t cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) d[i] = (TO)s[i];
}
template <typename TI>
__global__ void k_convert_in(const TI* __restrict__ s, double* __restrict__ d, int64_t cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) d[i] = (double)s[i];
}
hipError_t convert_f64(const double* src, void* dst, int64_t cnt, int to_f32, hipStream_t st) {
  if (cnt <= 0) return hipSuccess;
  if (to_f32)
    hipLaunchKernelGGL(k_convert<float>, dim3(nblk(cnt)), dim3(256), 0, st, src, (float*)dst, cnt);
  else
    hipLaunchKernelGGL(k_convert<double>, dim3(nblk(cnt)), dim3(256), 0, st, src, (double*)dst, cnt);
  return hipGetLastError();
}
hipError_t convert_to_f64(const void* src, double* dst, int64_t cnt, int from_f32, hipStream_t st) {
  if (cnt <= 0) return hipSuccess;
  if (from_f32)
    hipLaunchKernelGGL(k_convert_in<float>, dim3(nblk(cnt)), dim3(256), 0, st, (const float*)src, dst, cnt);
  else
    hipLaunchKernelGGL(k_convert_in<double>, dim3(nblk(cnt)), dim3(256), 0, st, (const double*)src, dst, cnt);
  return hipGetLastError();
}

template <typename TO>
__global__ void k_copy2d(const double* __restrict__ s, int64_t lds_, TO* __restrict__ d, int64_t ldd, int nr,
                         int nc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nr * nc) return;
  const int r = (int)(i / nc), c = (int)(i % nc);
  d[(int64_t)r * ldd + c] = (TO)s[(int64_t)r * lds_ + c];
}
hipError_t copy2d_f64_to(const double* src, int64_t lds_, void* dst, int64_t ldd, int nr, int nc, int to_f32,
                         hipStream_t st) {
  const int64_t cnt = (int64_t)nr * nc;
  if (cnt <= 0) return hipSuccess;
  if (to_f32)
    hipLaunchKernelGGL(k_copy2d<float>, dim3(nblk(cnt)), dim3(256), 0, st, src, lds_, (float*)dst, ldd, nr, nc);
  else
    hipLaunchKernelGGL(k_copy2d<double>, dim3(nblk(cnt)), dim3(256), 0, st, src, lds_, (double*)dst, ldd, nr,
                       nc);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------ K_N
// Neighbour p has offset (ox, oy) = (p / 2L - L + 1, p % 2L - L + 1) (lexicographic, ox major).
__device__ inline void offset_of(int p, int L, int& ox, int& oy) {
  ox = p / (2 * L) - L + 1;
  oy = p % (2 * L) - L + 1;
}

__global__ void __launch_bounds__(256) k_kn_factor(GridDev g, MaternDev mt, double* KN, double* LinvN,
                                                   int* status) {
  __shared__ double a[64][65];
  __shared__ int bad;
  const int M = g.M;
  const int tid = threadIdx.x;
  for (int attempt = 0; attempt < 2; ++attempt) {
    const double jit = attempt ? 1e-14 * mt.sigma2 * M : 0.0;
    if (tid == 0) bad = 0;
    for (int e = tid; e < M * M; e += 256) {
      const int p = e / M, q = e % M;
      int oxp, oyp, oxq, oyq;
      offset_of(p, g.L, oxp, oyp);
      offset_of(q, g.L, oxq, oyq);
      const double hx = (double)(oxp - oxq) * g.dx, hy = (double)(oyp - oyq) * g.dy;
      double v = matern_cov(sqrt(hx * hx + hy * hy), mt);
      if (p == q) v += jit;
      KN[e] = v;  // the matrix that is factored (weight refinement takes residuals against it)
      a[p][q] = v;
    }
    __syncthreads();
    for (int j = 0; j < M; ++j) {
      if (tid == 0) {
        const double d = a[j][j];
        if (!(d > 0.0)) {
          if (!bad) bad = j + 1;
          a[j][j] = 1.0;
        } else {
          a[j][j] = sqrt(d);
        }
      }
      __syncthreads();
      const double djj = a[j][j];
      for (int i = j + 1 + tid; i < M; i += 256) a[i][j] /= djj;
      __syncthreads();
      const int rem = M - 1 - j;
      for (int e = tid; e < rem * rem; e += 256) {
        const int i = j + 1 + e / rem, c = j + 1 + e % rem;
        if (c <= i) a[i][c] -= a[i][j] * a[c][j];
      }
      __syncthreads();
    }
    if (!bad) {
      if (tid == 0) *status = attempt;  // 0 = clean, 1 = jitter used
      break;
    }
    if (attempt == 1 && tid == 0) *status = -bad;
    __syncthreads();
  }
  __syncthreads();
  // inverse factor, one column per thread, straight to LinvN (row-major M x M)
  if (tid < M) {
    const int j = tid;
    for (int i = 0; i < j; ++i) LinvN[i * M + j] = 0.0;
    LinvN[j * M + j] = 1.0 / a[j][j];
    for (int i = j + 1; i < M; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += a[i][k] * LinvN[k * M + j];
      LinvN[i * M + j] = -s / a[i][i];
    }
  }
}

__global__ void k_kn_assemble(GridDev g, MaternDev mt, double* __restrict__ KN, double* __restrict__ A, double jit) {
  const int M = g.M;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * M) return;
  const int p = e / M, q = e % M;
  int oxp, oyp, oxq, oyq;
  offset_of(p, g.L, oxp, oyp);
  offset_of(q, g.L, oxq, oyq);
  const double hx = (double)(oxp - oxq) * g.dx, hy = (double)(oyp - oyq) * g.dy;
  const double v = matern_cov(sqrt(hx * hx + hy * hy), mt);
  const double a = p == q ? v + jit : v;
  if (KN) KN[e] = a;  // the matrix that is factored
  A[e] = a;
}

hipError_t kn_assemble(const GridDev& g, const MaternDev& mt, double* KN, double* A, double jit, hipStream_t st) {
  hipLaunchKernelGGL(k_kn_assemble, dim3(nblk((int64_t)g.M * g.M)), dim3(256), 0, st, g, mt, KN, A, jit);
  return hipGetLastError();
}

hipError_t kn_factor(const GridDev& g, const MaternDev& mt, double* KN, double* LinvN, int* status,
                     hipStream_t st) {
  if (g.M > 64) return hipErrorInvalidValue;  // one LDS tile; larger K_N go through the blocked path
  hipLaunchKernelGGL(k_kn_factor, dim3(1), dim3(256), 0, st, g, mt, KN, LinvN, status);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------ k_i and anchors
__global__ void k_site_kvec(GridDev g, MaternDev mt, const double* __restrict__ sites, int n,
                            int32_t* __restrict__ anchor, double* __restrict__ kvec) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * g.M) return;
  const int i = (int)(idx / g.M), p = (int)(idx % g.M);
  // cell of the site: t = (x - x0) / dx (IEEE division), i0 = floor(t), u = t - i0
  const double t = (sites[2 * i] - g.x0) / g.dx;
  const double s = (sites[2 * i + 1] - g.y0) / g.dy;
  int i0 = (int)floor(t), j0 = (int)floor(s);
  i0 = min(max(i0, 0), g.m1 - 1);
  j0 = min(max(j0, 0), g.m2 - 1);
  const double u = t - i0, v = s - j0;
  int ox, oy;
  offset_of(p, g.L, ox, oy);
  const double hx = ((double)ox - u) * g.dx, hy = ((double)oy - v) * g.dy;
  kvec[idx] = matern_cov(sqrt(hx * hx + hy * hy), mt);
  if (p == 0) {
    anchor[2 * i] = i0;
    anchor[2 * i + 1] = j0;
  }
}

hipError_t site_kvec(const GridDev& g, const MaternDev& mt, const double* sites, int n, int32_t* anchor,
                     double* kvec, hipStream_t st) {
  hipLaunchKernelGGL(k_site_kvec, dim3(nblk((int64_t)n * g.M)), dim3(256), 0, st, g, mt, sites, n, anchor, kvec);
  return hipGetLastError();
}

__global__ void k_transpose_w(const double* __restrict__ W, int n, int M, const int32_t* __restrict__ order,
                              double* __restrict__ Wt) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * M) return;
  const int s = (int)(idx % n), m = (int)(idx / n);
  const int i = order ? order[s] : s;
  Wt[idx] = W[(int64_t)i * M + m];
}
hipError_t transpose_w(const double* W, int n, int M, const int32_t* order, double* Wt, hipStream_t st) {
  hipLaunchKernelGGL(k_transpose_w, dim3(nblk((int64_t)n * M)), dim3(256), 0, st, W, n, M, order, Wt);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------ scans
// exclusive scan of int32 in[0..n) -> out[0..n], out[n] = total.  Three phases.
__global__ void __launch_bounds__(256) k_scan_blocks(const int32_t* in, int32_t* out, int n, int32_t* bsum) {
  __shared__ int32_t sh[256];
  const int base = blockIdx.x * 1024;
  int32_t v[4];
  int32_t loc = 0;
  for (int q = 0; q < 4; ++q) {
    const int i = base + threadIdx.x * 4 + q;
    v[q] = (i < n) ? in[i] : 0;
    loc += v[q];
  }
  sh[threadIdx.x] = loc;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele over thread totals
    const int32_t t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t run = sh[threadIdx.x] - loc;  // exclusive prefix of this thread
  for (int q = 0; q < 4; ++q) {
    const int i = base + threadIdx.x * 4 + q;
    if (i < n) out[i] = run;
    run += v[q];
  }
  if (threadIdx.x == 255) bsum[blockIdx.x] = sh[255];
}
__global__ void k_scan_bsum(int32_t* bsum, int nb, int32_t* out, int n) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t run = 0;
  for (int b = 0; b < nb; ++b) {
    const int32_t t = bsum[b];
    bsum[b] = run;
    run += t;
  }
  out[n] = run;
}
__global__ void k_scan_add(int32_t* out, int n, const int32_t* bsum) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += bsum[i / 1024];
}
static hipError_t scan_exclusive(const int32_t* in, int32_t* out, int n, int32_t* tmp, hipStream_t st) {
  const int nb = (n + 1023) / 1024;
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb > 0 ? nb : 1), dim3(256), 0, st, in, out, n, tmp);
  hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(64), 0, st, tmp, nb, out, n);
  hipLaunchKernelGGL(k_scan_add, dim3(nblk(n)), dim3(256), 0, st, out, n, tmp);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------ CSR build
__global__ void k_fill_i32(int32_t* p, int64_t cnt, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) p[i] = v;
}
__global__ void k_cell_count(const int32_t* anchor, int n, int m2, int32_t* cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[anchor[2 * i] * m2 + anchor[2 * i + 1]], 1);
}
__global__ void k_cell_fill(const int32_t* anchor, int n, int m2, const int32_t* ptr, int32_t* cur,
                            int32_t* sites) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = anchor[2 * i] * m2 + anchor[2 * i + 1];
  const int slot = atomicAdd(&cur[c], 1);
  sites[ptr[c] + slot] = i;
}
// slots were taken in arbitrary order; sorting each cell's (short) list by site
// index makes the layout deterministic
__global__ void k_cell_sort(int ncell, const int32_t* ptr, int32_t* sites) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int b = ptr[c], e = ptr[c + 1];
  for (int i = b + 1; i < e; ++i) {
    const int32_t v = sites[i];
    int j = i - 1;
    while (j >= b && sites[j] > v) {
      sites[j + 1] = sites[j];
      --j;
    }
    sites[j + 1] = v;
  }
}
// sites anchored at (i0, j0) touch padded nodes (i0 + L + ox, j0 + L + oy), ox, oy in
// [-L+1, L]; so node (p, r) collects anchors i0 in [p-2L, p-1], j0 in [r-2L, r-1].
__global__ void k_node_count(GridDev g, const int32_t* cell_cnt, int32_t* node_cnt) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.P1 * g.P2) return;
  const int p = q / g.P2, r = q % g.P2;
  int tot = 0;
  for (int i0 = max(p - 2 * g.L, 0); i0 <= min(p - 1, g.m1 - 1); ++i0)
    for (int j0 = max(r - 2 * g.L, 0); j0 <= min(r - 1, g.m2 - 1); ++j0) tot += cell_cnt[i0 * g.m2 + j0];
  node_cnt[q] = tot;
}
__global__ void k_node_fill(GridDev g, const int32_t* cell_ptr, const int32_t* cell_sites, const double* W,
                            const int32_t* node_ptr, int32_t* ent_site, double* ent_w) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.P1 * g.P2) return;
  const int p = q / g.P2, r = q % g.P2;
  int e = node_ptr[q];
  const int L2 = 2 * g.L;
  for (int i0 = max(p - 2 * g.L, 0); i0 <= min(p - 1, g.m1 - 1); ++i0)
    for (int j0 = max(r - 2 * g.L, 0); j0 <= min(r - 1, g.m2 - 1); ++j0) {
      const int c = i0 * g.m2 + j0;
      const int ox = p - g.L - i0, oy = r - g.L - j0;
      const int m = (ox + g.L - 1) * L2 + (oy + g.L - 1);
      for (int k = cell_ptr[c]; k < cell_ptr[c + 1]; ++k) {
        const int i = cell_sites[k];
        ent_site[e] = i;
        ent_w[e] = W[(int64_t)i * g.M + m];
        ++e;
      }
    }
}

hipError_t build_csr(const GridDev& g, const int32_t* anchor, const double* W, int n, const CsrWork& w,
                     int32_t* node_ptr, int32_t* ent_site, double* ent_w, hipStream_t st) {
  const int ncell = g.m1 * g.m2;
  const int nnode = g.P1 * g.P2;
  hipLaunchKernelGGL(k_fill_i32, dim3(nblk(ncell)), dim3(256), 0, st, w.cell_cnt, (int64_t)ncell, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(nblk(ncell)), dim3(256), 0, st, w.cell_cur, (int64_t)ncell, 0);
  hipLaunchKernelGGL(k_cell_count, dim3(nblk(n)), dim3(256), 0, st, anchor, n, g.m2, w.cell_cnt);
  hipError_t e = scan_exclusive(w.cell_cnt, w.cell_ptr, ncell, w.scan_tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_fill, dim3(nblk(n)), dim3(256), 0, st, anchor, n, g.m2, w.cell_ptr, w.cell_cur,
                     w.cell_sites);
  hipLaunchKernelGGL(k_cell_sort, dim3(nblk(ncell)), dim3(256), 0, st, ncell, w.cell_ptr, w.cell_sites);
  hipLaunchKernelGGL(k_node_count, dim3(nblk(nnode)), dim3(256), 0, st, g, w.cell_cnt, w.node_cnt);
  if ((e = scan_exclusive(w.node_cnt, node_ptr, nnode, w.scan_tmp, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_node_fill, dim3(nblk(nnode)), dim3(256), 0, st, g, w.cell_ptr, w.cell_sites, W, node_ptr,
                     ent_site, ent_w);
  return hipGetLastError();
}

// one thread per padded node: its entries keep their sites and order, only the weights change
__global__ void k_node_refill(GridDev g, const int32_t* __restrict__ anchor, const double* __restrict__ W,
                              const int32_t* __restrict__ node_ptr, const int32_t* __restrict__ ent_site,
                              double* __restrict__ ent_w) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.P1 * g.P2) return;
  const int p = q / g.P2, r = q % g.P2;
  const int L2 = 2 * g.L;
  for (int e = node_ptr[q]; e < node_ptr[q + 1]; ++e) {
    const int i = ent_site[e];
    const int ox = p - g.L - anchor[2 * i], oy = r - g.L - anchor[2 * i + 1];
    ent_w[e] = W[(int64_t)i * g.M + (ox + g.L - 1) * L2 + (oy + g.L - 1)];
  }
}

hipError_t refill_csr_weights(const GridDev& g, const int32_t* anchor, const double* W, const int32_t* node_ptr,
                              const int32_t* ent_site, double* ent_w, hipStream_t st) {
  const int nnode = g.P1 * g.P2;
  hipLaunchKernelGGL(k_node_refill, dim3(nblk(nnode)), dim3(256), 0, st, g, anchor, W, node_ptr, ent_site, ent_w);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------ scatter / gather
template <typename TS>
__global__ void k_scatter_image(int nnode, const int32_t* __restrict__ node_ptr,
                                const int32_t* __restrict__ ent_site, const double* __restrict__ ent_w,
                                const double* __restrict__ alpha, int64_t alpha_fs, TS* __restrict__ img,
                                int64_t img_fs) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (q >= nnode) return;
  const double* al = alpha + (int64_t)b * alpha_fs;
  double acc = 0.0;
  for (int e = node_ptr[q]; e < node_ptr[q + 1]; ++e) acc += al[ent_site[e]] * ent_w[e];
  img[(int64_t)b * img_fs + q] = (TS)acc;
}
hipError_t scatter_image(const GridDev& g, const int32_t* node_ptr, const int32_t* ent_site, const double* ent_w,
                         const double* alpha, int64_t alpha_fs, int B, void* img, int64_t img_fs, int to_f32,
                         hipStream_t st) {
  const int nnode = g.P1 * g.P2;
  dim3 grid(nblk(nnode), B);
  if (to_f32)
    hipLaunchKernelGGL(k_scatter_image<float>, grid, dim3(256), 0, st, nnode, node_ptr, ent_site, ent_w, alpha,
                       alpha_fs, (float*)img, img_fs);
  else
    hipLaunchKernelGGL(k_scatter_image<double>, grid, dim3(256), 0, st, nnode, node_ptr, ent_site, ent_w, alpha,
                       alpha_fs, (double*)img, img_fs);
  return hipGetLastError();
}

// site i in gather slot s (its transposed weights are column s of Wt)
template <typename TS>
__device__ inline double gather_one(const GridDev& g, const int32_t* anchor, const double* Wt, int n, int s,
                                    const TS* im, int64_t ldi) {
  const int i0 = anchor[2 * s], j0 = anchor[2 * s + 1];
  const int L2 = 2 * g.L;
  double acc = 0.0;
  // loads of sixteen neighbours are issued together; the sum runs in the order of m
  for (int m0 = 0; m0 < g.M; m0 += 16) {
    double wv[16], iv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int m = m0 + u;
      wv[u] = 0.0;
      iv[u] = 0.0;
      if (m < g.M) {
        const int ox = m / L2 - g.L + 1, oy = m % L2 - g.L + 1;
        wv[u] = Wt[(int64_t)m * n + s];
        iv[u] = (double)im[(int64_t)(i0 + g.L + ox) * ldi + (j0 + g.L + oy)];
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (m0 + u < g.M) acc += wv[u] * iv[u];
  }
  return acc;
}

// Adjoint gather (the transpose of Steps 5-6): out[b][i] = sum_m W[i][m] img[b][node(i, m)].
// Four lanes per site, lane q taking m = q, q+4, ... (M = 4 L^2, so L^2 terms each, with
// L a compile-time constant so the neighbour offsets fold): every lane's loads go out
// together, its partial runs in the order of m, and the four partials are added as
// (q0 + q1) + (q2 + q3).
template <typename TS, int L>
__global__ void __launch_bounds__(256) k_gather_sites(GridDev g, const int32_t* __restrict__ anchor,
                                                      const double* __restrict__ Wt,
                                                      const int32_t* __restrict__ order, int n,
                                                      const TS* __restrict__ img, int64_t img_fs, int64_t ldi,
                                                      double* __restrict__ out, int64_t out_fs) {
  constexpr int L2 = 2 * L, PER = L * L;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = t >> 2, q = t & 3;  // gather slot, quarter of the neighbourhood
  const int b = blockIdx.y;
  const bool ok = s < n;  // all four lanes of a site agree; no early exit before the shuffles
  const int ss = ok ? s : 0;
  const int ii = order ? order[ss] : ss;  // needed only for the store
  const TS* base = img + (int64_t)b * img_fs + (int64_t)(anchor[2 * ss] + L) * ldi + (anchor[2 * ss + 1] + L);
  double wv[PER], iv[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int m = q + 4 * u;  // q is a lane value: the offsets below are q-dependent but cheap
    const int ox = m / L2 - L + 1, oy = m % L2 - L + 1;
    wv[u] = ok ? Wt[(int64_t)m * n + ss] : 0.0;
    iv[u] = ok ? (double)base[(int64_t)ox * ldi + oy] : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < PER; ++u) acc += wv[u] * iv[u];
  const double o1 = __shfl_xor(acc, 1);
  const double pair = (q & 1) ? o1 + acc : acc + o1;  // (q0 + q1) or (q2 + q3), on both lanes of a pair
  const double o2 = __shfl_xor(pair, 2);
  const double tot = (q & 2) ? o2 + pair : pair + o2;
  if (ok && q == 0) out[(int64_t)b * out_fs + ii] = tot;
}

template <typename TS>
__global__ void __launch_bounds__(256) k_gather_generic(GridDev g, const int32_t* __restrict__ anchor,
                                                        const double* __restrict__ Wt,
                                                        const int32_t* __restrict__ order, int n,
                                                        const TS* __restrict__ img, int64_t img_fs, int64_t ldi,
                                                        double* __restrict__ out, int64_t out_fs) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (s >= n) return;
  const int i = order ? order[s] : s;
  out[(int64_t)b * out_fs + i] = gather_one<TS>(g, anchor, Wt, n, s, img + (int64_t)b * img_fs, ldi);
}

template <typename TS>
hipError_t gather_launch(const GridDev& g, const int32_t* anchor, const double* Wt, const int32_t* order, int n,
                         const TS* img, int64_t img_fs, int64_t ldi, int B, double* out, int64_t out_fs,
                         hipStream_t st) {
  dim3 grid((unsigned)((4 * (int64_t)n + 255) / 256), B);
  switch (g.L) {
    case 1: hipLaunchKernelGGL((k_gather_sites<TS, 1>), grid, dim3(256), 0, st, g, anchor, Wt, order, n, img, img_fs, ldi, out, out_fs); break;
    case 2: hipLaunchKernelGGL((k_gather_sites<TS, 2>), grid, dim3(256), 0, st, g, anchor, Wt, order, n, img, img_fs, ldi, out, out_fs); break;
    case 3: hipLaunchKernelGGL((k_gather_sites<TS, 3>), grid, dim3(256), 0, st, g, anchor, Wt, order, n, img, img_fs, ldi, out, out_fs); break;
    case 4: hipLaunchKernelGGL((k_gather_sites<TS, 4>), grid, dim3(256), 0, st, g, anchor, Wt, order, n, img, img_fs, ldi, out, out_fs); break;
    default:  // L > 4: one thread per site and field, neighbours sixteen at a time
      hipLaunchKernelGGL(k_gather_generic<TS>, dim3((unsigned)((n + 255) / 256), B), dim3(256), 0, st, g, anchor, Wt,
                         order, n, img, img_fs, ldi, out, out_fs);
      break;
  }
  return hipGetLastError();
}

hipError_t gather_sites(const GridDev& g, const int32_t* anchor, const double* Wt, const int32_t* order, int n,
                        const void* img, int64_t img_fs, int64_t ldi, int B, int from_f32, double* out,
                        int64_t out_fs, hipStream_t st) {
  if (from_f32)
    return gather_launch<float>(g, anchor, Wt, order, n, (const float*)img, img_fs, ldi, B, out, out_fs, st);
  return gather_launch<double>(g, anchor, Wt, order, n, (const double*)img, img_fs, ldi, B, out, out_fs, st);
}

// residual of conditional simulation: out[r][i] = y[i] - (u_r(s_i) + sd * xi_{r,i})
template <typename TS>
__global__ void k_csim_residual(GridDev g, const int32_t* __restrict__ anchor, const double* __restrict__ Wt,
                                const int32_t* __restrict__ order, int n, const TS* __restrict__ img,
                                int64_t img_fs, int64_t ldi, const double* __restrict__ y, double sd, uint32_t k0,
                                uint32_t k1, int r0, double* __restrict__ out, int64_t out_fs) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (s >= n) return;
  const int i = order ? order[s] : s;
  const double us = gather_one<TS>(g, anchor, Wt, n, s, img + (int64_t)r * img_fs, ldi);
  u32x4 c;
  c.v[0] = (uint32_t)i;
  c.v[1] = (uint32_t)(r0 + r);
  c.v[2] = STREAM_NUGGET;
  c.v[3] = 0;
  const u32x4 w = philox4x32_10(c, k0, k1);
  double n0, n1;
  box_muller_f64(w.v[0], w.v[1], n0, n1);
  out[(int64_t)r * out_fs + i] = y[i] - (us + sd * n0);
}
hipError_t csim_residual(const GridDev& g, const int32_t* anchor, const double* Wt, const int32_t* order, int n,
                         const void* img, int64_t img_fs, int64_t ldi, int R, int from_f32, const double* y,
                         double noise_sd, uint64_t seed, int r0, double* out, int64_t out_fs, hipStream_t st) {
  dim3 grid(nblk(n), R);
  const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
  if (from_f32)
    hipLaunchKernelGGL(k_csim_residual<float>, grid, dim3(256), 0, st, g, anchor, Wt, order, n, (const float*)img,
                       img_fs, ldi, y, noise_sd, k0, k1, r0, out, out_fs);
  else
    hipLaunchKernelGGL(k_csim_residual<double>, grid, dim3(256), 0, st, g, anchor, Wt, order, n,
                       (const double*)img, img_fs, ldi, y, noise_sd, k0, k1, r0, out, out_fs);
  return hipGetLastError();
}

}  // namespace krig

namespace krig {

// per-block min, max and count of negatives of a FP64 array (host finishes)
__global__ void __launch_bounds__(256) k_minmax(const double* __restrict__ x, int64_t cnt, double* bmin,
                                                double* bmax, int* bneg) {
  __shared__ double smin[256], smax[256];
  __shared__ int sneg[256];
  double mn = 1e300, mx = -1e300;
  int ng = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[i];
    mn = fmin(mn, v);
    mx = fmax(mx, v);
    ng += v < 0.0;
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  sneg[threadIdx.x] = ng;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
      sneg[threadIdx.x] += sneg[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bmin[blockIdx.x] = smin[0];
    bmax[blockIdx.x] = smax[0];
    bneg[blockIdx.x] = sneg[0];
  }
}

hipError_t minmax_blocks(const double* x, int64_t cnt, double* bmin, double* bmax, int* bneg, int nblocks,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_minmax, dim3(nblocks), dim3(256), 0, st, x, cnt, bmin, bmax, bneg);
  return hipGetLastError();
}

// x <- sqrt(max(x, 0) * scale)
__global__ void k_sqrt_clamp(double* x, int64_t cnt, double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) x[i] = sqrt(fmax(x[i], 0.0) * scale);
}

hipError_t sqrt_clamp(double* x, int64_t cnt, double scale, hipStream_t st) {
  hipLaunchKernelGGL(k_sqrt_clamp, dim3(nblk(cnt)), dim3(256), 0, st, x, cnt, scale);
  return hipGetLastError();
}

// x <- x / d, element by element
__global__ void k_div(double* x, const double* d, int64_t cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) x[i] = x[i] / d[i];
}

hipError_t div_f64(double* x, const double* d, int64_t cnt, hipStream_t st) {
  hipLaunchKernelGGL(k_div, dim3(nblk(cnt)), dim3(256), 0, st, x, d, cnt);
  return hipGetLastError();
}

}  // namespace krig
