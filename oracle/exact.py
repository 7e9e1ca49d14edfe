"""Exact Kriging, Section 2 (eqs. findc and predictionh).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The data are residuals y = z - X beta_hat (the linear part is handled outside
the prediction step, Section 2), so the coefficients are
    c = M^{-1} y,   M = K + tau^2 I,                               eq. (findc)
obtained from a Cholesky factorisation and two triangular solves (the route the
paper names right after eq. predictionf), and the prediction at any location is
    g_hat(s) = sum_i k(s, s_i) c_i.                                eq. (predictionh)
"""
from __future__ import annotations

import numpy as np
from scipy import linalg

from .matern import Matern


def kriging_matrix(sites: np.ndarray, kern: Matern) -> np.ndarray:
    """M = K + tau^2 I with K_il = k(s_i, s_l) (Section 2, before eq. findbeta)."""
    K = kern.cross(sites, sites)
    K[np.diag_indices_from(K)] += kern.tau2
    return K


class ExactKriging:
    """Cholesky factor of M, reused for many right-hand sides."""

    def __init__(self, sites: np.ndarray, kern: Matern):
        self.sites = np.asarray(sites, dtype=np.float64)
        self.kern = kern
        self.M = kriging_matrix(self.sites, kern)
        self.cho = linalg.cho_factor(self.M, lower=True, check_finite=True)

    def coef(self, y: np.ndarray) -> np.ndarray:
        """c = M^{-1} y (eq. findc); y may be (n,) or (B, n)."""
        y = np.asarray(y, dtype=np.float64)
        if y.ndim == 1:
            return linalg.cho_solve(self.cho, y)
        return linalg.cho_solve(self.cho, y.T).T

    def predict_at(self, pts: np.ndarray, c: np.ndarray, chunk: int = 4096) -> np.ndarray:
        """g_hat(s_j) = sum_i k(s_j, s_i) c_i for each row of pts (eq. predictionh)."""
        pts = np.asarray(pts, dtype=np.float64)
        out = np.empty(pts.shape[0])
        for s in range(0, pts.shape[0], chunk):
            out[s:s + chunk] = self.kern.cross(pts[s:s + chunk], self.sites) @ c
        return out

    def std_error(self, pts: np.ndarray) -> np.ndarray:
        """Kriging standard error sqrt(sigma^2 - k(s)^T M^{-1} k(s)) of g at pts.

        This is the conditional standard deviation of g(s) given the data under
        the model of eq. (ObservationalModel); conditional simulation must
        reproduce it (Section 5.1, the ensemble-vs-exact comparison).
        """
        pts = np.asarray(pts, dtype=np.float64)
        kx = self.kern.cross(self.sites, pts)          # n x p
        v = linalg.cho_solve(self.cho, kx)
        var = self.kern.sigma2 - np.einsum("ij,ij->j", kx, v)
        return np.sqrt(np.maximum(var, 0.0))

    def grad_y(self, pts: np.ndarray, g: np.ndarray) -> np.ndarray:
        """Gradient of sum_j g_j * g_hat(s_j) w.r.t. y: M^{-1} K(obs, grid) g."""
        pts = np.asarray(pts, dtype=np.float64)
        v = self.kern.cross(self.sites, pts) @ np.asarray(g, dtype=np.float64)
        return linalg.cho_solve(self.cho, v)


def gp_draw(sites: np.ndarray, kern: Matern, rng: np.random.Generator,
            nugget: bool = True, jitter: float = 1e-12) -> np.ndarray:
    """An exact draw of g at the sites (plus N(0, tau^2) noise if nugget).

    This is the data-generating model of eq. (ObservationalModel) with X beta = 0.
    """
    K = kern.cross(sites, sites)
    K[np.diag_indices_from(K)] += jitter * kern.sigma2
    Lc = np.linalg.cholesky(K)
    g = Lc @ rng.standard_normal(len(sites))
    if nugget and kern.tau2 > 0:
        g = g + np.sqrt(kern.tau2) * rng.standard_normal(len(sites))
    return g
