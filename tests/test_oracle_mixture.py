"""Pins of the spatially weighted mixture of stationary components (CPU only)."""
import numpy as np

from oracle.matern import Matern
from oracle.mixture import mixture_cov, mixture_exact, mixture_rapid
from oracle.rapid import Grid, RapidPredictor


def setup(seed=0, n=50, m=29, L=2):
    g = Grid(m, m, 0.0, 0.0, 1.0 / (m - 1), 1.0 / (m - 1), L)
    rng = np.random.default_rng(seed)
    return g, rng.uniform(0.0, 1.0, (n, 2)), rng.standard_normal(n)


def comps2():
    k1, k2 = Matern(1.0, 0.3, 1.5), Matern(0.5, 0.12, 2.5)
    lam1 = lambda p: np.cos(1.2 * p[..., 0]) ** 2 + 0.1
    lam2 = lambda p: np.sin(1.2 * p[..., 0]) ** 2 + 0.1
    return [(k1, lam1), (k2, lam2)]


def test_single_unit_component_is_the_stationary_predictor():
    g, sites, alpha = setup()
    k = Matern(1.0, 0.3, 1.5)
    one = lambda p: np.ones(p.shape[:-1])
    got = mixture_rapid(g, [(k, one)], sites, alpha)
    ref = RapidPredictor(g, k, sites).predict_direct(alpha).reshape(g.m1, g.m2)
    assert np.array_equal(got, ref)


def test_mixture_covariance_is_symmetric_and_positive_definite():
    _, sites, _ = setup(1, n=120)
    K = mixture_cov(comps2())(sites[:, None, :], sites[None, :, :])
    assert np.allclose(K, K.T, rtol=0, atol=1e-15)
    assert np.linalg.eigvalsh(K).min() > -1e-12 * np.abs(K).max()


def test_rapid_mixture_approximates_the_exact_mixture_and_is_linear():
    g, sites, alpha = setup(2, n=60, m=41, L=3)
    comps = comps2()
    got = mixture_rapid(g, comps, sites, alpha)
    ref = mixture_exact(comps, sites, alpha, g.nodes()).reshape(g.m1, g.m2)
    # each component is a stationary rapid prediction; the error is theirs (L = 3)
    assert np.abs(got - ref).max() < 1e-3 * np.abs(ref).max()
    a2 = np.random.default_rng(9).standard_normal(len(alpha))
    lin = mixture_rapid(g, comps, sites, 2.0 * alpha - a2)
    assert np.allclose(lin, 2.0 * got - mixture_rapid(g, comps, sites, a2), rtol=0, atol=1e-12 * np.abs(got).max())
