"""Nonstationary covariance vectors with the stationary grid interpolation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 6 (discussion) extends the rapid predictor to a nonstationary covariance:
Step 3's covariance vector k_i between site i and its neighbourhood nodes may come
from the nonstationary covariance, while Step 4 still interpolates it with the
stationary K_N, and the convolution still uses the stationary lag image.  The
coefficients alpha then come from the caller's (nonstationary) kriging system.

Reading: k_i[m] = C(g_m, s_i) for the neighbour nodes g_m of site i in the offset
order of `rapid.offsets`; A_i = K_N^{-1} k_i exactly as in `rapid.neighbour_weights`.
"""
from __future__ import annotations

import numpy as np
from scipy import linalg

from .matern import Matern
from .rapid import Grid, kn_matrix, offsets, site_cells


def neighbour_nodes(grid: Grid, sites: np.ndarray) -> np.ndarray:
    """Coordinates of every site's M neighbourhood nodes, n x M x 2 (offset order)."""
    i0, j0, _, _ = site_cells(grid, sites)
    off = offsets(grid.L)
    gx = grid.x0 + (i0[:, None] + off[None, :, 0]) * grid.dx
    gy = grid.y0 + (j0[:, None] + off[None, :, 1]) * grid.dy
    return np.stack([gx, gy], axis=2)


def kvecs_cov(grid: Grid, sites: np.ndarray, cov) -> np.ndarray:
    """k_i[m] = cov(g_m, s_i) for a covariance function cov(p, q) of two point arrays
    (... x 2 each, broadcasting), n x M."""
    sites = np.asarray(sites, dtype=np.float64)
    g = neighbour_nodes(grid, sites)
    return cov(g, np.broadcast_to(sites[:, None, :], g.shape))


def weights_from_kvec(grid: Grid, kern: Matern, kvec: np.ndarray) -> np.ndarray:
    """Step 4 with a given k_i: A_i = K_N^{-1} k_i (Cholesky solve, one jitter retry as
    in rapid.neighbour_weights), n x M."""
    KN = kn_matrix(grid, kern)
    try:
        cho = linalg.cho_factor(KN, lower=True)
    except linalg.LinAlgError:
        cho = linalg.cho_factor(KN + 1e-14 * kern.sigma2 * grid.M * np.eye(grid.M), lower=True)
    return linalg.cho_solve(cho, np.asarray(kvec, dtype=np.float64).T).T


def scaled_cov(kern: Matern, sd):
    """A nonstationary covariance: C(p, q) = sd(p) sd(q) k(p - q), with sd a positive
    function of a point array (... x 2) -- a valid covariance for any stationary k."""
    def cov(p, q):
        h = p - q
        return sd(p) * sd(q) * kern.of_lag(h[..., 0], h[..., 1])
    return cov


def exact_ns_prediction(cov, tau2: float, sites: np.ndarray, y: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Exact kriging with covariance cov: (C(pts, sites)) (C(sites, sites) + tau2 I)^{-1} y
    (eqs. findc and predictionh with the nonstationary covariance)."""
    sites = np.asarray(sites, dtype=np.float64)
    K = cov(sites[:, None, :], sites[None, :, :]) + tau2 * np.eye(len(sites))
    alpha = linalg.cho_solve(linalg.cho_factor(K, lower=True), y)
    return cov(pts[:, None, :], sites[None, :, :]) @ alpha, alpha
