"""Matern covariance, eq. (Matern1) of Section 3 ("Approximation Error").

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper writes k(s, s') = sigma^2 * phi(alpha * ||s - s'||) with
phi(d) = d^nu K_nu(d) / (2^(nu-1) Gamma(nu)) and calls alpha the "scale (range)"
parameter.  Its numerical examples (range 0.25 on the unit square, range 1.21
in degrees for the rainfall fit) and the remark that doubling the range is the
same interpolation problem as doubling the spacing only make sense when the
range divides the distance, so this oracle reads the covariance as
    k(d) = sigma^2 * phi(d / rho),   rho = range,
with no sqrt(2 nu) factor (the paper's phi has none).
"""
from __future__ import annotations

import numpy as np
from scipy import special


def phi_general(d, nu: float) -> np.ndarray:
    """phi(d) = d^nu K_nu(d) / (2^(nu-1) Gamma(nu)), eq. (Matern1); phi(0) = 1.

    Uses the modified Bessel function of the second kind from SciPy (a library
    routine).  Valid for any nu > 0.
    """
    d = np.asarray(d, dtype=np.float64)
    out = np.ones_like(d)
    pos = d > 0
    dp = d[pos]
    out[pos] = dp ** nu * special.kv(nu, dp) / (2.0 ** (nu - 1.0) * special.gamma(nu))
    return out


def phi_closed(d, nu: float) -> np.ndarray:
    """Elementary closed forms of phi for half-integer smoothness.

    For nu = p + 1/2 the Bessel function K_nu is elementary, which gives
        nu = 1/2 : exp(-d)
        nu = 3/2 : (1 + d) exp(-d)
        nu = 5/2 : (1 + d + d^2/3) exp(-d)
    (pinned against phi_general in the test suite).
    """
    d = np.asarray(d, dtype=np.float64)
    e = np.exp(-d)
    if nu == 0.5:
        return e
    if nu == 1.5:
        return (1.0 + d) * e
    if nu == 2.5:
        return (1.0 + d + d * d / 3.0) * e
    raise ValueError(f"no closed form for nu={nu}")


def phi(d, nu: float) -> np.ndarray:
    """phi of eq. (Matern1): closed form for nu in {1/2, 3/2, 5/2}, else Bessel."""
    if nu in (0.5, 1.5, 2.5):
        return phi_closed(d, nu)
    return phi_general(d, nu)


class Matern:
    """Stationary isotropic Matern covariance k(s, s') = sigma2 * phi(||s-s'|| / rho).

    tau2 is the nugget variance of eq. (ObservationalModel); it enters only the
    kriging system M = K + tau2 I of eq. (findc), never the covariance k itself
    (k is the covariance of the latent field g).
    """

    def __init__(self, sigma2: float, rho: float, nu: float, tau2: float = 0.0):
        if sigma2 <= 0 or rho <= 0 or nu <= 0 or tau2 < 0:
            raise ValueError("invalid Matern parameters")
        self.sigma2 = float(sigma2)
        self.rho = float(rho)
        self.nu = float(nu)
        self.tau2 = float(tau2)

    def of_dist(self, d) -> np.ndarray:
        """k as a function of the Euclidean distance d."""
        return self.sigma2 * phi(np.asarray(d, dtype=np.float64) / self.rho, self.nu)

    def of_lag(self, hx, hy) -> np.ndarray:
        """k as a function of a lag vector (hx, hy) (stationarity, Section 2.1)."""
        hx = np.asarray(hx, dtype=np.float64)
        hy = np.asarray(hy, dtype=np.float64)
        return self.of_dist(np.sqrt(hx * hx + hy * hy))

    def cross(self, a: np.ndarray, b: np.ndarray) -> np.ndarray:
        """Dense covariance matrix k(a_i, b_j) for point sets a (p x 2), b (q x 2)."""
        a = np.asarray(a, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        hx = a[:, 0:1] - b[None, :, 0]
        hy = a[:, 1:2] - b[None, :, 1]
        return self.of_lag(hx, hy)
