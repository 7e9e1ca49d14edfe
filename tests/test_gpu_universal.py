"""GPU: universal kriging with a GLS trend (krig_predict_universal) against the oracle."""
import sys

import numpy as np
import pytest

import workloads as wl
from parity_bars import BAR_F32, bar_for, check
from oracle.exact import ExactKriging
from oracle.matern import Matern
from oracle.rapid import Grid, RapidPredictor
from oracle.universal import gls, universal_rapid

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def relmax(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def design(pts):
    return np.stack([np.ones(len(pts)), pts[:, 0], pts[:, 1], pts[:, 0] * pts[:, 1]], 1)


@pytest.fixture(scope="module")
def small():
    w = wl.small_field()
    g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
    k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
    return w, g, k, RapidPredictor(g, k, w.sites), ExactKriging(w.sites, k)


def plan_with_oracle_weights(krig, w, rp, dtype):
    p = krig.plan_for(w, dtype)
    p.set_weights(dev(np.stack([rp.i0, rp.j0], 1), torch.int32), dev(rp.W))
    return p


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_universal_matches_oracle(krig, small, dtype):
    w, g, k, rp, ek = small
    say("universal kriging small field", dtype)
    p = plan_with_oracle_weights(krig, w, rp, dtype)
    X = design(w.sites)
    Xg = design(g.nodes()).T.reshape(4, g.m1, g.m2)
    rng = np.random.default_rng(0)
    z = np.stack([w.y[0] + X @ [2.0, -1.0, 0.5, 3.0], rng.standard_normal(w.n) + X @ [0.0, 1.0, 1.0, 0.0]])
    beta = torch.empty(2, 4, dtype=torch.float64, device="cuda:0")
    coef = torch.empty(2, w.n, dtype=torch.float64, device="cuda:0")
    got = host(p.predict_universal(dev(z), dev(X.T), dev(Xg), beta_out=beta, coef_out=coef))
    B_, C_ = host(beta), host(coef)
    for b in range(2):
        bref, cref = gls(ek, X, z[b])
        # GLS through the GPU's explicit inverse factor vs the oracle's Cholesky solves
        assert relmax(B_[b], bref) < 1e-9
        assert relmax(C_[b], cref) < 1e-9
        ref = universal_rapid(ek, rp, X, Xg, z[b])
        check(f"universal kriging field {b} {dtype}", relmax(got[b], ref), 1e-10 if dtype == "f64" else BAR_F32)
    again = host(p.predict_universal(dev(z), dev(X.T), dev(Xg)))
    assert np.array_equal(got, again)


def test_universal_trend_only_data(krig, small):
    w, g, k, rp, ek = small
    say("universal kriging, data in the trend space")
    p = plan_with_oracle_weights(krig, w, rp, "f64")
    X = design(w.sites)
    nodes = g.nodes()
    Xg = design(nodes).T.reshape(4, g.m1, g.m2)
    bt = np.array([0.7, -1.2, 2.0, 0.4])
    beta = torch.empty(1, 4, dtype=torch.float64, device="cuda:0")
    coef = torch.empty(1, w.n, dtype=torch.float64, device="cuda:0")
    got = host(p.predict_universal(dev((X @ bt)[None]), dev(X.T), dev(Xg), beta_out=beta, coef_out=coef))
    assert np.allclose(host(beta)[0], bt, rtol=0, atol=1e-8)
    assert np.abs(host(coef)).max() < 1e-6
    assert np.abs(got[0] - (design(nodes) @ bt).reshape(g.m1, g.m2)).max() < 1e-8


def test_universal_dependent_covariates_and_errors(krig, small):
    w, g, k, rp, ek = small
    say("universal kriging, dependent covariates and argument errors")
    p = krig.plan_for(w, "f64")
    X = design(w.sites)
    Xd = np.concatenate([X, X[:, 1:2] * 2.0], 1)  # a column repeated: X^T M^{-1} X singular
    Xg = design(g.nodes()).T.reshape(4, g.m1, g.m2)
    Xgd = np.concatenate([Xg, 2.0 * Xg[1:2]], 0)
    got = host(p.predict_universal(dev(w.y), dev(Xd.T), dev(Xgd)))
    assert np.all(np.isnan(got))
    for npc in (0, 17):
        Xs = dev(np.ones((npc, w.n)))
        Xgr = dev(np.ones((npc, g.m1, g.m2)))
        out = p.empty(1, g.m1, g.m2)
        assert p.lib.krig_predict_universal(p.h, 1, dev(w.y).data_ptr(), npc, Xs.data_ptr(), Xgr.data_ptr(),
                                            out.data_ptr(), None, None) == -1
