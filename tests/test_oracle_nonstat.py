"""Pins of the nonstationary covariance-vector path (CPU only)."""
import numpy as np

from oracle.matern import Matern
from oracle.nonstat import exact_ns_prediction, kvecs_cov, neighbour_nodes, scaled_cov, weights_from_kvec
from oracle.rapid import Grid, RapidPredictor, kn_matrix, kvecs, neighbour_weights, rapid_direct, site_cells


def setup(seed=0, n=60, m=33, L=2):
    g = Grid(m, m, 0.0, 0.0, 1.0 / (m - 1), 1.0 / (m - 1), L)
    rng = np.random.default_rng(seed)
    sites = rng.uniform(0.0, 1.0, (n, 2))
    return g, Matern(1.0, 0.3, 1.5, 1e-3), sites


def test_stationary_covariance_reduces_to_the_standard_weights():
    g, k, sites = setup()
    kv = kvecs_cov(g, sites, scaled_cov(k, lambda p: np.ones(p.shape[:-1])))
    _, _, u, v = site_cells(g, sites)
    assert np.allclose(kv, kvecs(g, k, u, v), rtol=0, atol=1e-15)
    _, _, W = neighbour_weights(g, k, sites)
    assert np.array_equal(weights_from_kvec(g, k, kv), W)


def test_neighbour_nodes_and_interpolation_residual():
    g, k, sites = setup(1)
    nodes = neighbour_nodes(g, sites)
    # every site lies in the central cell of its 2L x 2L neighbourhood
    assert np.all(nodes[:, 0, 0] <= sites[:, 0]) and np.all(nodes[:, -1, 0] >= sites[:, 0])
    sd = lambda p: 1.0 + 0.5 * np.sin(3.0 * p[..., 0]) * np.cos(2.0 * p[..., 1])
    kv = kvecs_cov(g, sites, scaled_cov(k, sd))
    W = weights_from_kvec(g, k, kv)
    assert np.abs(W @ kn_matrix(g, k) - kv).max() < 1e-12  # eq. weights with the given k_i


def test_ns_approximation_improves_as_the_covariance_nears_the_stationary_one():
    # rapid NS prediction (NS k_i, stationary K_N and lag) vs exact NS kriging with the
    # same coefficients: the paper expects accuracy when the nonstationary covariance is
    # close to a stationary one, so the error must shrink with the amplitude of the sd
    # variation, down to the stationary approximation error (L = 2, coarse mesh) at 0
    g, k, sites = setup(2, n=80, m=41)
    rng = np.random.default_rng(3)
    y = rng.standard_normal(len(sites))
    rp = RapidPredictor(g, k, sites)
    nodes = g.nodes()
    errs = []
    for amp in (0.4, 0.1, 0.0):
        sd = lambda p, a=amp: 1.0 + a * np.sin(2.0 * p[..., 0] + 1.0) * np.cos(1.5 * p[..., 1])
        cov = scaled_cov(k, sd)
        ref, alpha = exact_ns_prediction(cov, k.tau2, sites, y, nodes)
        W = weights_from_kvec(g, k, kvecs_cov(g, sites, cov))
        rq = RapidPredictor(g, k, sites)
        rq.W = W
        rq.A = rq.A.__class__((W.ravel(), rq.A.indices, rq.A.indptr), shape=rq.A.shape)
        got = rapid_direct(g, k, rq.cstar(alpha))
        errs.append(np.abs(got - ref).max() / np.abs(ref).max())
    assert errs[0] > 3 * errs[1] > 9 * errs[2] and errs[2] < 0.05, errs
