"""Conditional simulation with the rapid predictor (Section 1, steps (1)-(2); Section 6).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conditional simulation (CS) draws an unconditional field, then kriges the
residual between the data and the simulated data and adds the result:
    field = u_grid + g_hat(y - (u_sites + tau * xi)).
The paper draws u on the grid by circulant embedding (discussion section) and
at the sites by the local simulation of Bailey et al., which it does not
specify; here u at the sites is read off the simulated padded grid with the
same M-neighbour weights that define the rapid predictor,
    u(s_i) = sum_m W[i, m] u[anchor_i + offset_m].

Circulant embedding (Dietrich & Newsam): embed the covariance of the padded
P1 x P2 node set in an Fs1 x Fs2 torus with minimal-image lags
(Fs >= 2(P-1)), take its eigenvalues Lambda = FFT2(first row) (real), and form
    Y = FFT2( sqrt(Lambda / (Fs1 Fs2)) * (xi1 + i xi2) );
Re Y and Im Y are two independent draws with the embedded covariance.  The
embedding can have small negative eigenvalues when the range is large
relative to the torus (the paper's caveat); the reading used here clamps them
to zero when min(Lambda) >= -1e-6 max(Lambda) and otherwise enlarges the torus:
both axes move to their next even 2^a 3^b size, up to twice the first size
(`ce_torus`); beyond that the embedding fails.
"""
from __future__ import annotations

import numpy as np

from . import philox
from .exact import ExactKriging
from .matern import Matern
from .rapid import Grid, RapidPredictor, fft_len, offsets, lag_quadrant, rapid_fft

CE_CLAMP_TOL = 1e-6
CE_MAX_GROWTH = 2


class CEFailure(ValueError):
    """The circulant embedding has eigenvalues below -CE_CLAMP_TOL of the largest."""


def ce_eigs(grid: Grid, kern: Matern, Fs1: int, Fs2: int):
    """Eigenvalues of the circulant embedding of the padded-grid covariance.

    Returns (Lambda clamped at 0, number of clamped entries, min/max ratio).
    Raises ValueError when the most negative eigenvalue exceeds the tolerance.
    """
    if Fs1 < 2 * (grid.P1 - 1) or Fs2 < 2 * (grid.P2 - 1):
        raise ValueError("embedding torus too small")
    u = np.arange(Fs1)
    w = np.arange(Fs2)
    du = np.minimum(u, Fs1 - u) * grid.dx
    dw = np.minimum(w, Fs2 - w) * grid.dy
    c = kern.of_lag(du[:, None], dw[None, :])
    lam = np.fft.fft2(c).real
    lmax = lam.max()
    lmin = lam.min()
    if lmin < -CE_CLAMP_TOL * lmax:
        raise CEFailure("circulant embedding not non-negative definite")
    nclamp = int(np.sum(lam < 0))
    return np.maximum(lam, 0.0), nclamp, lmin / lmax


def ce_torus(grid: Grid, kern: Matern):
    """The embedding torus (Fs1, Fs2): the smallest even 2^a 3^b sizes >= 2(P - 1) per axis,
    then, while the embedding fails the clamp tolerance, both axes at their next even 2^a 3^b
    size, up to CE_MAX_GROWTH times the first sizes.  Raises CEFailure when none qualifies."""
    F10 = fft_len(2 * (grid.P1 - 1))
    F20 = fft_len(2 * (grid.P2 - 1))
    F1, F2 = F10, F20
    while F1 <= CE_MAX_GROWTH * F10 and F2 <= CE_MAX_GROWTH * F20:
        try:
            ce_eigs(grid, kern, F1, F2)
            return F1, F2
        except CEFailure:
            F1, F2 = fft_len(F1 + 1), fft_len(F2 + 1)
    raise CEFailure(f"no torus up to {CE_MAX_GROWTH}x ({F10} x {F20}) embeds the covariance")


def ce_pair(lam: np.ndarray, seed: int, pair: int, P1: int, P2: int):
    """Two unconditional padded-grid fields (realisations 2*pair, 2*pair+1)."""
    Fs1, Fs2 = lam.shape
    eps = philox.ce_noise(seed, pair, Fs1, Fs2)
    Y = np.fft.fft2(np.sqrt(lam / (Fs1 * Fs2)) * eps)
    return Y.real[:P1, :P2].copy(), Y.imag[:P1, :P2].copy()


def site_values(grid: Grid, u_img: np.ndarray, i0, j0, W) -> np.ndarray:
    """u(s_i) = sum_m W[i, m] u[i0+L+ox_m, j0+L+oy_m] (the same weights as the predictor)."""
    off = offsets(grid.L)
    p = i0[:, None] + grid.L + off[None, :, 0]
    q = j0[:, None] + grid.L + off[None, :, 1]
    return np.sum(W * u_img[p, q], axis=1)


class ConditionalSimulator:
    """Oracle CS: exact FP64 pieces, rapid predictor through the FP64 FFT variant."""

    def __init__(self, grid: Grid, kern: Matern, sites: np.ndarray, Fs1: int, Fs2: int):
        self.grid = grid
        self.kern = kern
        self.rp = RapidPredictor(grid, kern, sites)
        self.ek = ExactKriging(sites, kern)
        self.lam, self.nclamp, self.ratio = ce_eigs(grid, kern, Fs1, Fs2)
        self.lag = lag_quadrant(grid, kern)

    def realisation(self, seed: int, r: int, y: np.ndarray) -> np.ndarray:
        """Conditional realisation r (0-based) on the m1 x m2 grid."""
        g = self.grid
        ure, uim = ce_pair(self.lam, seed, r // 2, g.P1, g.P2)
        u = ure if r % 2 == 0 else uim
        us = site_values(g, u, self.rp.i0, self.rp.j0, self.rp.W)
        ys = us + np.sqrt(self.kern.tau2) * philox.nugget_noise(seed, r, len(us))
        c = self.ek.coef(np.asarray(y, dtype=np.float64) - ys)
        pred = rapid_fft(g, self.lag, self.rp.cstar(c))
        return u[g.L:g.L + g.m1, g.L:g.L + g.m2] + pred
