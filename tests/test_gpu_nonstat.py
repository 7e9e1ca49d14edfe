"""GPU: weights from caller (nonstationary) covariance vectors, krig_set_kvec."""
import sys

import numpy as np
import pytest

import workloads as wl
from parity_bars import BAR_F32, bar_for, check, weight_residual_ratio
from oracle.matern import Matern
from oracle.nonstat import kvecs_cov, scaled_cov, weights_from_kvec
from oracle.rapid import Grid, cstar_image, kn_matrix, kvecs, rapid_direct, site_cells, sparse_A

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


def sd(p):
    return 1.0 + 0.3 * np.sin(3.0 * p[..., 0] + 0.5) * np.cos(2.0 * p[..., 1])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_set_kvec_small_field(krig, dtype):
    w = wl.small_field()
    g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
    k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
    say("set_kvec small field", dtype)
    p = krig.plan_for(w, dtype)
    kv = kvecs_cov(g, w.sites, scaled_cov(k, sd))
    p.set_kvec(dev(kv))
    anc, W = p.weights()
    anc, W = host(anc).astype(np.int64), host(W)
    check(f"set_kvec small field: weights vs oracle {dtype}", np.abs(W - weights_from_kvec(g, k, kv)).max(), 1e-9)
    # eq. weights with the caller's k_i
    check(f"set_kvec small field: residual / backward-stable bound {dtype}",
          weight_residual_ratio(W, kn_matrix(g, k), kv), 1.0)
    # predictions from caller coefficients use the new weights (oracle with the same W)
    alpha = np.random.default_rng(0).standard_normal((2, w.n))
    yh = host(p.convolve(dev(alpha)))
    A = sparse_A(g, anc[:, 0], anc[:, 1], W)
    for b in range(2):
        ref = rapid_direct(g, k, cstar_image(g, A, alpha[b])).reshape(g.m1, g.m2)
        check(f"set_kvec small field: prediction field {b} {dtype}", relmax(yh[b], ref), bar_for(dtype))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_set_kvec_refill_matches_a_rebuilt_structure(krig, dtype):
    # set_kvec rewrites only the weights of the scatter structure; a plan given the same
    # weights through set_weights rebuilds the structure from scratch: same layout, same
    # order, so the scatter image and the predictions agree bit for bit
    w = wl.paper_field()
    g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
    k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
    say("set_kvec refill vs rebuilt structure, paper field", dtype)
    p = krig.plan_for(w, dtype)
    p.set_kvec(dev(kvecs_cov(g, w.sites, scaled_cov(k, sd))))
    anc, W = p.weights()
    q = krig.plan_for(w, dtype)
    q.set_weights(anc, W)
    alpha = dev(np.random.default_rng(5).standard_normal((3, w.n)))
    assert np.array_equal(host(p.scatter(alpha)), host(q.scatter(alpha)))
    assert np.array_equal(host(p.convolve(alpha)), host(q.convolve(alpha)))
    gup = torch.ones(3, w.m1, w.m2, dtype=p.tdtype, device="cuda:0")
    dp, _ = p.adjoint(gup, alpha=alpha, want_dlag=False)
    dq, _ = q.adjoint(gup, alpha=alpha, want_dlag=False)
    assert np.array_equal(host(dp), host(dq))


def test_set_kvec_stationary_reproduces_the_plan(krig):
    w = wl.small_field()
    g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
    k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
    say("set_kvec with the stationary k_i")
    p = krig.plan_for(w, "f64")
    _, W0 = p.weights()
    W0 = host(W0)
    y = dev(w.y)
    before = host(p.predict(y))
    _, _, u, v = site_cells(g, w.sites)
    p.set_kvec(dev(kvecs(g, k, u, v)))
    _, W1 = p.weights()
    # the plan evaluated k_i on the GPU, this call takes the oracle's FP64 values: the
    # last-bit differences pass through K_N^{-1} (the stationary weights test's bar)
    assert np.abs(host(W1) - W0).max() < 1e-9
    assert relmax(host(p.predict(y)), before) < 1e-12


def test_set_kvec_paper_field_residual(krig):
    w = wl.paper_field()
    g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
    k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
    say("set_kvec paper field (K_N cond ~3e13)")
    p = krig.plan_for(w, "f32")
    kv = kvecs_cov(g, w.sites, scaled_cov(k, sd))
    p.set_kvec(dev(kv))
    _, W = p.weights()
    # K_N is ill-conditioned: the weights are checked through the interpolation residual,
    # against the bound of a backward-stable solve
    check("set_kvec paper field: residual / backward-stable bound",
          weight_residual_ratio(host(W), kn_matrix(g, k), kv), 1.0)
    with pytest.raises(TypeError):
        p.set_kvec(dev(kv, torch.float32))
