"""Universal kriging: a linear trend in covariates estimated by GLS (eqs. findbeta,
findc, predictionf), with the spatial part predicted exactly or by the rapid method.

TEST INFRASTRUCTURE ONLY (see the package docstring).

    beta_hat = (X^T M^{-1} X)^{-1} X^T M^{-1} z      (eq. findbeta)
    c        = M^{-1} (z - X beta_hat)                (eq. findc)
    f_hat_j  = X_j beta_hat + g_hat(s_j)              (eq. predictionf)

X is n x p (row i: the covariates at site i); the covariates at the prediction
points are given the same way.  M^{-1} is applied through the Cholesky factor.
"""
from __future__ import annotations

import numpy as np
from scipy import linalg

from .exact import ExactKriging


def gls(ek: ExactKriging, X: np.ndarray, z: np.ndarray):
    """(beta_hat, c) for one data vector z (n,) and covariates X (n x p)."""
    X = np.asarray(X, dtype=np.float64)
    MiX = ek.coef(X.T).T                 # M^{-1} X, n x p
    Miz = ek.coef(z)
    beta = linalg.solve(X.T @ MiX, X.T @ Miz, assume_a="pos")
    return beta, ek.coef(z - X @ beta)


def universal_exact(ek: ExactKriging, X: np.ndarray, Xp: np.ndarray, z: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """f_hat at pts with covariates Xp (npts x p) at those points, spatial part exact."""
    beta, c = gls(ek, X, z)
    return Xp @ beta + ek.predict_at(pts, c)


def universal_rapid(ek: ExactKriging, rp, X: np.ndarray, Xgrid: np.ndarray, z: np.ndarray) -> np.ndarray:
    """f_hat on the m1 x m2 grid: Xgrid (p x m1 x m2) beta_hat + the rapid prediction of c."""
    beta, c = gls(ek, X, z)
    g = rp.grid
    return np.tensordot(beta, Xgrid, axes=1) + rp.predict_direct(c).reshape(g.m1, g.m2)
