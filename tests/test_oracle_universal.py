"""Pins of universal kriging (GLS trend, eqs. findbeta / findc / predictionf), CPU only."""
import numpy as np

from oracle.exact import ExactKriging
from oracle.matern import Matern
from oracle.rapid import Grid, RapidPredictor
from oracle.universal import gls, universal_exact, universal_rapid


def setup(seed=0, n=70, m=33, L=3):
    g = Grid(m, m, 0.0, 0.0, 1.0 / (m - 1), 1.0 / (m - 1), L)
    rng = np.random.default_rng(seed)
    sites = rng.uniform(0.0, 1.0, (n, 2))
    k = Matern(1.0, 0.25, 1.5, 0.05)
    return g, k, sites, rng


def design(pts):
    return np.stack([np.ones(len(pts)), pts[:, 0], pts[:, 1], pts[:, 0] * pts[:, 1]], 1)


def test_trend_only_data_is_reproduced_exactly():
    # z = X beta (in the trend space): GLS returns beta, c = 0, and the prediction is the trend
    g, k, sites, rng = setup()
    ek = ExactKriging(sites, k)
    beta = np.array([0.7, -1.2, 2.0, 0.4])
    X = design(sites)
    b, c = gls(ek, X, X @ beta)
    assert np.allclose(b, beta, rtol=0, atol=1e-10) and np.abs(c).max() < 1e-9
    nodes = g.nodes()
    f = universal_exact(ek, X, design(nodes), X @ beta, nodes)
    assert np.allclose(f, design(nodes) @ beta, rtol=0, atol=1e-9)


def test_gls_matches_whitened_least_squares_and_residual_is_orthogonal():
    # beta_hat solves the least-squares problem of the whitened system L^{-1} X b ~ L^{-1} z
    # (numpy's lstsq, an independent route), and X^T c = X^T M^{-1}(z - X beta) = 0
    g, k, sites, rng = setup(1)
    ek = ExactKriging(sites, k)
    X = design(sites)
    z = rng.standard_normal(len(sites)) + X @ [1.0, 0.5, -0.3, 0.2]
    b, c = gls(ek, X, z)
    Lc = np.linalg.cholesky(ek.M)
    ref = np.linalg.lstsq(np.linalg.solve(Lc, X), np.linalg.solve(Lc, z), rcond=None)[0]
    assert np.allclose(b, ref, rtol=1e-10, atol=1e-12)
    assert np.abs(X.T @ c).max() < 1e-9 * np.abs(c).sum()


def test_without_covariates_is_simple_kriging_and_rapid_tracks_exact():
    g, k, sites, rng = setup(2)
    ek = ExactKriging(sites, k)
    z = rng.standard_normal(len(sites))
    b, c = gls(ek, np.zeros((len(sites), 0)), z)
    assert b.shape == (0,) and np.allclose(c, ek.coef(z), rtol=0, atol=1e-14)
    X = design(sites)
    nodes = g.nodes()
    rp = RapidPredictor(g, k, sites)
    Xg = design(nodes).T.reshape(4, g.m1, g.m2)
    fr = universal_rapid(ek, rp, X, Xg, z + X @ [0.3, 1.0, -1.0, 0.5])
    fe = universal_exact(ek, X, design(nodes), z + X @ [0.3, 1.0, -1.0, 0.5], nodes).reshape(g.m1, g.m2)
    # the trend is exact on both sides; the spatial part carries the rapid approximation error (L = 3)
    assert np.abs(fr - fe).max() < 1e-3 * np.abs(fe).max()
