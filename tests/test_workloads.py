"""The shared input generators: shapes, determinism, and the RFF draw's covariance."""
import numpy as np

import workloads as wl
from oracle.matern import Matern


def test_generators_are_seeded_and_shaped():
    a = wl.small_field()
    b = wl.small_field()
    assert a.sites.shape == (200, 2) and a.y.shape == (1, 200)
    assert np.array_equal(a.sites, b.sites) and np.array_equal(a.y, b.y)
    p = wl.paper_field()
    assert p.sites.shape == (1368, 2)
    assert p.sites[:, 0].min() >= 0 and p.sites[:, 0].max() <= 2 and p.sites[:, 1].max() <= 1
    assert (p.m1, p.m2, p.L) == (350, 350, 3) and np.isclose(p.dx, 2 / 349) and np.isclose(p.dy, 1 / 349)
    gb = wl.grad_batch()
    assert gb.y.shape == (16, 1368) and gb.extra["mask"].shape == (350, 350)
    assert np.array_equal(gb.sites, p.sites)


def test_rff_draw_has_matern_covariance():
    # empirical covariance of many RFF draws at a few lags vs the oracle's Matern
    rng = np.random.default_rng(0)
    pts = np.array([[0.0, 0.0], [0.05, 0.0], [0.1, 0.05], [0.3, 0.2]])
    for nu, rho in ((0.5, 0.2), (1.5, 0.1), (2.5, 0.3)):
        f = wl.rff_draw(rng, pts, 1.0, rho, nu, nfeat=256, count=3000)
        C = (f.T @ f) / f.shape[0]
        K = Matern(1.0, rho, nu).cross(pts, pts)
        assert np.abs(C - K).max() < 0.08, (nu, np.abs(C - K).max())
