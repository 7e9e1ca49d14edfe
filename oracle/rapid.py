"""The rapid approximate predictor, Section 2.2 ("Rapid prediction algorithm").

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation (the paper's, with the readings used where it is silent or garbled):

* Prediction grid: m1 x m2 nodes s_(a,b) = (x0 + a dx, y0 + b dy), a < m1,
  b < m2, both end points included.  The paper asks for odd m1, m2; oddness
  plays no role in a zero-padded linear convolution and is not required here.
* Padding: the grid is extended by L nodes on every side, giving the padded
  grid of P1 = m1 + 2L by P2 = m2 + 2L nodes (padded index = unpadded + L), so
  that every site has its full neighbourhood (Section 2.2, around Figure 1; the
  paper's worked example of the padding is arithmetically inconsistent, so the
  symmetric L-node padding is used).
* Neighbourhood N(i): the 2L x 2L square of nodes whose central box holds the
  site, i.e. offsets (ox, oy) in {-L+1, ..., L}^2 from the lower-left corner
  (i0, j0) of the cell holding the site, M = (2L)^2.  The offsets are listed in
  one fixed lexicographic order (ox major) for every site, as the remark after
  Step 7 requires for a single K_N.
* Cell of a site: t = (x - x0)/dx, i0 = floor(t), u = t - i0 (same in y).  A
  site on a cell edge takes the lower/left cell (floor).  Sites must satisfy
  0 <= t <= m1 - 1 (inside the grid's bounding box).
* Outputs: the predictions are the m1 x m2 unpadded nodes (padded indices
  L .. L+m-1), the "first m1 x m2 block" of Step 7 after the padding shift.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import linalg, sparse

from .matern import Matern


@dataclass(frozen=True)
class Grid:
    m1: int
    m2: int
    x0: float
    y0: float
    dx: float
    dy: float
    L: int

    @property
    def M(self) -> int:
        return (2 * self.L) ** 2

    @property
    def P1(self) -> int:
        return self.m1 + 2 * self.L

    @property
    def P2(self) -> int:
        return self.m2 + 2 * self.L

    def nodes(self) -> np.ndarray:
        """Unpadded prediction nodes, row-major over (a, b): (m1*m2) x 2."""
        a = self.x0 + np.arange(self.m1) * self.dx
        b = self.y0 + np.arange(self.m2) * self.dy
        X, Y = np.meshgrid(a, b, indexing="ij")
        return np.stack([X.ravel(), Y.ravel()], axis=1)

    def padded_node(self, p, q):
        """Coordinates of padded node (p, q) (p, q may be arrays)."""
        return (self.x0 + (np.asarray(p) - self.L) * self.dx,
                self.y0 + (np.asarray(q) - self.L) * self.dy)


def offsets(L: int) -> np.ndarray:
    """The M = (2L)^2 neighbour offsets (ox, oy) in lexicographic, ox-major order."""
    r = np.arange(-L + 1, L + 1)
    ox, oy = np.meshgrid(r, r, indexing="ij")
    return np.stack([ox.ravel(), oy.ravel()], axis=1)


def kn_matrix(grid: Grid, kern: Matern) -> np.ndarray:
    """K_N: covariances among the M neighbourhood nodes (Step 1 / eq. weights).

    Identical for every site because k is stationary (remark after eq. weights).
    """
    off = offsets(grid.L).astype(np.float64)
    hx = (off[:, 0:1] - off[None, :, 0]) * grid.dx
    hy = (off[:, 1:2] - off[None, :, 1]) * grid.dy
    return kern.of_lag(hx, hy)


def site_cells(grid: Grid, sites: np.ndarray):
    """Anchor node (i0, j0) and in-cell fractions (u, v) of every site.

    Raises ValueError for a site outside the grid's bounding box.
    """
    sites = np.asarray(sites, dtype=np.float64)
    t = (sites[:, 0] - grid.x0) / grid.dx
    s = (sites[:, 1] - grid.y0) / grid.dy
    if np.any(t < 0) or np.any(t > grid.m1 - 1) or np.any(s < 0) or np.any(s > grid.m2 - 1):
        raise ValueError("site outside the prediction grid")
    i0 = np.floor(t).astype(np.int64)
    j0 = np.floor(s).astype(np.int64)
    return i0, j0, t - i0, s - j0


def kvecs(grid: Grid, kern: Matern, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """k_i (Step 3): covariance of each site with its M neighbours, n x M.

    The site sits at (u dx, v dy) from its anchor node; neighbour p sits at
    (ox_p dx, oy_p dy), so the lag is ((ox_p - u) dx, (oy_p - v) dy).
    """
    off = offsets(grid.L).astype(np.float64)
    hx = (off[None, :, 0] - u[:, None]) * grid.dx
    hy = (off[None, :, 1] - v[:, None]) * grid.dy
    return kern.of_lag(hx, hy)


def neighbour_weights(grid: Grid, kern: Matern, sites: np.ndarray):
    """Steps 1, 3, 4: A_i = K_N^{-1} k_i for every site (eq. weights).

    K_N^{-1} is applied through its Cholesky factor and two triangular solves
    (mathematically the explicit inverse of Step 1, numerically the stable
    route: K_N is badly conditioned for smooth kernels).  If the factorisation
    fails, it is retried once with jitter on the diagonal.  Returns
    (i0, j0, W) with W of shape n x M in the offset order of `offsets`.
    """
    i0, j0, u, v = site_cells(grid, sites)
    KN = kn_matrix(grid, kern)
    try:
        cho = linalg.cho_factor(KN, lower=True)
    except linalg.LinAlgError:
        # reading used where the paper only notes the instability of smooth kernels:
        # one retry with jitter 1e-14 * sigma^2 * M on the diagonal
        cho = linalg.cho_factor(KN + 1e-14 * kern.sigma2 * grid.M * np.eye(grid.M), lower=True)
    kv = kvecs(grid, kern, u, v)                       # n x M
    W = linalg.cho_solve(cho, kv.T).T
    return i0, j0, W


def neighbour_columns(grid: Grid, i0: np.ndarray, j0: np.ndarray) -> np.ndarray:
    """Padded-grid node index (row-major over P1 x P2) of every (site, neighbour)."""
    off = offsets(grid.L)
    p = i0[:, None] + grid.L + off[None, :, 0]
    q = j0[:, None] + grid.L + off[None, :, 1]
    return p * grid.P2 + q


def sparse_A(grid: Grid, i0: np.ndarray, j0: np.ndarray, W: np.ndarray) -> sparse.csr_matrix:
    """The sparse n x (P1 P2) interpolation matrix A of eq. (ApproxCovarianceGeneral)."""
    n = W.shape[0]
    cols = neighbour_columns(grid, i0, j0)
    rows = np.repeat(np.arange(n), W.shape[1])
    return sparse.csr_matrix((W.ravel(), (rows, cols.ravel())), shape=(n, grid.P1 * grid.P2))


def cstar_image(grid: Grid, A: sparse.csr_matrix, c: np.ndarray) -> np.ndarray:
    """Step 5: c* = A^T c, reshaped to the padded P1 x P2 image (Step 6).

    c may be (n,) or (B, n); the result is (P1, P2) or (B, P1, P2).
    """
    c = np.asarray(c, dtype=np.float64)
    if c.ndim == 1:
        return (A.T @ c).reshape(grid.P1, grid.P2)
    return np.stack([(A.T @ ci).reshape(grid.P1, grid.P2) for ci in c])


def rapid_direct(grid: Grid, kern: Matern, cimg: np.ndarray, out_idx=None,
                 chunk_elems: int = 1 << 24) -> np.ndarray:
    """g_approx(s_j) = sum_q phi(s_j - s_q) c*_q by a DIRECT sum (eq. ApproxPrediction2).

    cimg is one padded P1 x P2 image.  out_idx selects unpadded output nodes
    as flat indices a*m2 + b (default: all m1*m2).  Only the nonzero entries of
    c* contribute.  This is the convolution of eq. (Convolution) written out.
    """
    cimg = np.asarray(cimg, dtype=np.float64)
    if out_idx is None:
        out_idx = np.arange(grid.m1 * grid.m2)
    out_idx = np.asarray(out_idx)
    a = out_idx // grid.m2
    b = out_idx % grid.m2
    sx = grid.x0 + a * grid.dx
    sy = grid.y0 + b * grid.dy
    pq = np.nonzero(cimg)
    cx, cy = grid.padded_node(pq[0], pq[1])
    cv = cimg[pq]
    out = np.zeros(len(out_idx))
    step = max(1, chunk_elems // max(1, len(cv)))
    for s in range(0, len(out_idx), step):
        hx = sx[s:s + step, None] - cx[None, :]
        hy = sy[s:s + step, None] - cy[None, :]
        out[s:s + step] = kern.of_lag(hx, hy) @ cv
    return out


def lag_quadrant(grid: Grid, kern: Matern) -> np.ndarray:
    """The filter Phi of Step 2 on its non-negative lags: (m1+L) x (m2+L).

    lag[a, b] = k((a dx, b dy)); these are all the lags that occur between an
    unpadded output node and a padded source node.
    """
    a = np.arange(grid.m1 + grid.L) * grid.dx
    b = np.arange(grid.m2 + grid.L) * grid.dy
    return kern.of_lag(a[:, None], b[None, :])


def conv_lag_direct(grid: Grid, lag: np.ndarray, cimg: np.ndarray) -> np.ndarray:
    """y[a, b] = sum_{p,q} lag[|a+L-p|, |b+L-q|] c*[p, q] over unpadded (a, b).

    The same linear convolution as `rapid_direct`, but with the filter given as
    an arbitrary lag quadrant (used for gradients w.r.t. the lag image and for
    the FFT pins).  Direct O(N nnz) sum.
    """
    cimg = np.asarray(cimg, dtype=np.float64)
    pq = np.nonzero(cimg)
    cv = cimg[pq]
    A = np.arange(grid.m1)[:, None] + grid.L - pq[0][None, :]     # m1 x nnz
    Bq = np.arange(grid.m2)[:, None] + grid.L - pq[1][None, :]    # m2 x nnz
    out = np.zeros((grid.m1, grid.m2))
    for a in range(grid.m1):
        vals = lag[np.abs(A[a])[None, :], np.abs(Bq)]              # m2 x nnz
        out[a] = vals @ cv
    return out


def fft_len(need: int) -> int:
    """Smallest even 2^a 3^b >= need (any size >= need gives the same result)."""
    best = None
    p2 = 2
    while p2 < 4 * need:
        p3 = p2
        while p3 < 4 * need:
            if p3 >= need and (best is None or p3 < best):
                best = p3
            p3 *= 3
        p2 *= 2
    return best


def embed_even(lag: np.ndarray, F1: int, F2: int) -> np.ndarray:
    """Circulant embedding Phi~ of Step 2: even reflection of the lag quadrant.

    Entry (u, w) holds lag[min(u, F1-u), min(w, F2-w)] where that lag lies in
    the quadrant, zero elsewhere (those entries never reach a kept output).
    """
    n1, n2 = lag.shape
    E = np.zeros((F1, F2))
    u = np.arange(F1)
    w = np.arange(F2)
    du = np.minimum(u, F1 - u)
    dw = np.minimum(w, F2 - w)
    ok1 = du < n1
    ok2 = dw < n2
    E[np.ix_(ok1, ok2)] = lag[np.ix_(du[ok1], dw[ok2])]
    return E


def rapid_fft(grid: Grid, lag: np.ndarray, cimg: np.ndarray) -> np.ndarray:
    """Step 7 with numpy's FP64 FFT (TEST-ONLY variant for full large grids).

    C~ holds c* in its leading P1 x P2 block; the kept outputs are rows/cols
    L .. L+m-1.  Validated against the direct sum in the test suite.
    """
    F1 = fft_len(grid.m1 + grid.P1 - 1)
    F2 = fft_len(grid.m2 + grid.P2 - 1)
    E = embed_even(lag, F1, F2)
    C = np.zeros((F1, F2))
    C[:grid.P1, :grid.P2] = cimg
    Y = np.fft.ifft2(np.fft.fft2(E) * np.fft.fft2(C)).real
    return Y[grid.L:grid.L + grid.m1, grid.L:grid.L + grid.m2]


def filter_spectrum_reflected(lag: np.ndarray, F1: int, F2: int) -> np.ndarray:
    """Step 2's filter spectrum: the 2-D DFT of the even reflection of the lag quadrant (real,
    F1 x F2).  TEST-ONLY FFT form, as rapid_fft uses it."""
    return np.fft.fft2(embed_even(lag, F1, F2)).real


def filter_spectrum_centered(grid: Grid, kern: Matern, F1: int, F2: int) -> np.ndarray:
    """The alternative filter set-up of the remark after Step 7, which avoids the reflections at
    the price of one more FFT: evaluate the covariance between the torus centre node
    (F1/2, F2/2) and every torus node from plain coordinate differences, take its 2-D DFT and
    divide by the DFT of the indicator of the centre node (which removes the centre's phase).
    Every lag up to half the torus is filled, so the middle of the filter image differs from
    the reflected quadrant's zeros; those lags never reach a kept output (reading of Step 2)."""
    r = (np.arange(F1) - F1 // 2) * grid.dx
    c = (np.arange(F2) - F2 // 2) * grid.dy
    img = kern.of_lag(r[:, None], c[None, :])
    delta = np.zeros((F1, F2))
    delta[F1 // 2, F2 // 2] = 1.0
    return np.fft.fft2(img) / np.fft.fft2(delta)


def rapid_fft_spectrum(grid: Grid, spec: np.ndarray, cimg: np.ndarray) -> np.ndarray:
    """Step 7 with a given F1 x F2 filter spectrum (numpy FP64 FFT, TEST-ONLY): the kept
    outputs of ifft2(spec * fft2(C~))."""
    F1, F2 = spec.shape
    C = np.zeros((F1, F2))
    C[:grid.P1, :grid.P2] = cimg
    Y = np.fft.ifft2(spec * np.fft.fft2(C)).real
    return Y[grid.L:grid.L + grid.m1, grid.L:grid.L + grid.m2]


class RapidPredictor:
    """Steps 1-7 for one site set: weights once, then many coefficient vectors."""

    def __init__(self, grid: Grid, kern: Matern, sites: np.ndarray):
        self.grid = grid
        self.kern = kern
        self.sites = np.asarray(sites, dtype=np.float64)
        self.i0, self.j0, self.W = neighbour_weights(grid, kern, self.sites)
        self.A = sparse_A(grid, self.i0, self.j0, self.W)

    def cstar(self, c):
        return cstar_image(self.grid, self.A, c)

    def predict_direct(self, c, out_idx=None):
        """One coefficient vector c -> predictions at the selected nodes."""
        return rapid_direct(self.grid, self.kern, self.cstar(c), out_idx)

    def predict_fft(self, c):
        """Full m1 x m2 predictions via the test-only FP64 FFT variant."""
        return rapid_fft(self.grid, lag_quadrant(self.grid, self.kern), self.cstar(c))

    def approx_kernel(self, i: int, pts: np.ndarray) -> np.ndarray:
        """k_approx(s, s_i) = sum_q k(s, s_q) A_iq at arbitrary pts (eq. ApproxCovarianceGeneral)."""
        g = self.grid
        off = offsets(g.L)
        p = self.i0[i] + g.L + off[:, 0]
        q = self.j0[i] + g.L + off[:, 1]
        nx, ny = g.padded_node(p, q)
        nodes = np.stack([nx, ny], axis=1)
        return self.kern.cross(pts, nodes) @ self.W[i]


def grid_unit(m1: int, m2: int, L: int, xlen: float = 1.0, ylen: float = 1.0,
              x0: float = 0.0, y0: float = 0.0) -> Grid:
    """A grid whose m1 x m2 nodes span [x0, x0+xlen] x [y0, y0+ylen], ends included."""
    return Grid(m1, m2, x0, y0, xlen / (m1 - 1), ylen / (m2 - 1), L)


def fill_distance_of_grid(grid: Grid) -> float:
    """delta for a regular grid (Section 3.2): half the cell diagonal."""
    return 0.5 * math.hypot(grid.dx, grid.dy)
