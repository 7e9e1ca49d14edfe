"""Nonstationary covariance as a spatially weighted sum of stationary components.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 6 (discussion): a nonstationary covariance that is a combination of several
stationary covariances with weights varying over space is predicted by running the
rapid predictor for each stationary component and combining the results with the
spatial weight functions.  Reading:

    C(s, s') = sum_c lam_c(s) lam_c(s') k_c(s - s')        (a valid covariance)
    yhat(s)  = sum_i C(s, s_i) alpha_i
             = sum_c lam_c(s) * [ sum_i k_c(s - s_i) (lam_c(s_i) alpha_i) ]

so each component is a stationary prediction of the coefficients lam_c(s_i) alpha_i,
weighted by lam_c on the grid.  The rapid form replaces each bracket by the rapid
predictor of component c (its own weights and lag image).
"""
from __future__ import annotations

import numpy as np

from .rapid import Grid, RapidPredictor, rapid_direct


def mixture_cov(comps):
    """C(p, q) for comps = [(kern_c, lam_c)], lam_c a function of a point array (... x 2)."""
    def cov(p, q):
        h = p - q
        return sum(lam(p) * lam(q) * k.of_lag(h[..., 0], h[..., 1]) for k, lam in comps)
    return cov


def mixture_exact(comps, sites: np.ndarray, alpha: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """sum_i C(pts, s_i) alpha_i with the mixture covariance (dense, small cases)."""
    sites = np.asarray(sites, dtype=np.float64)
    return mixture_cov(comps)(pts[:, None, :], sites[None, :, :]) @ alpha


def mixture_rapid(grid: Grid, comps, sites: np.ndarray, alpha: np.ndarray, predictors=None) -> np.ndarray:
    """The rapid form on the m1 x m2 grid: sum_c lam_c(node) * rapid_c(lam_c(s_i) alpha_i).
    predictors: optional RapidPredictor per component (to supply given weights)."""
    sites = np.asarray(sites, dtype=np.float64)
    nodes = grid.nodes()
    out = np.zeros(grid.m1 * grid.m2)
    for c, (k, lam) in enumerate(comps):
        rp = predictors[c] if predictors is not None else RapidPredictor(grid, k, sites)
        beta = lam(sites) * alpha
        out += lam(nodes) * rapid_direct(grid, k, rp.cstar(beta))
    return out.reshape(grid.m1, grid.m2)
