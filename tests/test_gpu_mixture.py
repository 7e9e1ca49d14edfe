"""GPU: the nonstationary mixture of stationary components (krig_mixture)."""
import dataclasses
import sys

import numpy as np
import pytest

import workloads as wl
from parity_bars import BAR_F32, bar_for, check
from oracle.matern import Matern
from oracle.mixture import mixture_rapid
from oracle.rapid import Grid, RapidPredictor

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


def lam1(p):
    return np.cos(2.0 * p[..., 0]) ** 2 + 0.1


def lam2(p):
    return np.sin(2.0 * p[..., 0]) ** 2 + 0.1


def components(w, shared):
    """The workload's own kernel and a second, smoother and shorter-range one: with the same
    neighbour order L (one transform geometry: the fused path, the coefficient scaling in the
    scatter and the weighted sum in one inverse-row pass) or with L + 1 (separate component
    images and a combine pass)."""
    w2 = dataclasses.replace(w, sigma2=0.5, rho=0.6 * w.rho, nu=2.5, L=w.L if shared else w.L + 1)
    return [(w, lam1), (w2, lam2)]


@pytest.mark.parametrize("shared", [True, False], ids=["same-L", "different-L"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_mixture_matches_oracle(krig, dtype, shared):
    w = wl.small_field()
    g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
    say("mixture of two components, small field", dtype, "same L" if shared else "different L")
    comps = components(w, shared)
    plans, ocomps, preds = [], [], []
    for wc, lam in comps:
        k = Matern(wc.sigma2, wc.rho, wc.nu, wc.tau2)
        gc = Grid(wc.m1, wc.m2, wc.x0, wc.y0, wc.dx, wc.dy, wc.L)
        rp = RapidPredictor(gc, k, wc.sites)
        p = krig.plan_for(wc, dtype)
        p.set_weights(dev(np.stack([rp.i0, rp.j0], 1), torch.int32), dev(rp.W))  # identical weights
        plans.append(p)
        ocomps.append((k, lam))
        preds.append(rp)
    alpha = np.random.default_rng(0).standard_normal((2, w.n))
    nodes = g.nodes()
    lam_sites = np.stack([lam(w.sites) for _, lam in comps])
    lam_grid = np.stack([lam(nodes).reshape(w.m1, w.m2) for _, lam in comps])
    got = host(krig.mixture(plans, dev(alpha), dev(lam_sites), dev(lam_grid)))
    for b in range(2):
        # the oracle's components run on their own grids' L (each plan's neighbourhood)
        ref = np.zeros((w.m1, w.m2))
        for (k, lam), rp in zip(ocomps, preds):
            ref += lam(nodes).reshape(w.m1, w.m2) * rp.predict_direct(lam(w.sites) * alpha[b]).reshape(w.m1, w.m2)
        check(f"mixture field {b} {dtype} {'same' if shared else 'different'} L", relmax(got[b], ref), bar_for(dtype))
    again = host(krig.mixture(plans, dev(alpha), dev(lam_sites), dev(lam_grid)))
    assert np.array_equal(got, again)


def test_mixture_single_unit_component_is_the_convolution(krig):
    w = wl.small_field()
    say("mixture with one unit component")
    p = krig.plan_for(w, "f32")
    alpha = dev(np.random.default_rng(1).standard_normal((3, w.n)))
    ref = host(p.convolve(alpha))
    got = host(krig.mixture([p], alpha, dev(np.ones((1, w.n))), dev(np.ones((1, w.m1, w.m2)))))
    assert np.array_equal(got, ref)


def test_mixture_argument_errors(krig):
    w = wl.small_field()
    say("mixture argument errors")
    p = krig.plan_for(w, "f64")
    other = krig.plan_for(dataclasses.replace(w, x0=w.x0 - w.dx, m1=w.m1 + 1), "f64")  # another grid
    f32 = krig.plan_for(w, "f32")
    alpha = dev(np.zeros((1, w.n)))
    ones = lambda C: (dev(np.ones((C, w.n))), dev(np.ones((C, w.m1, w.m2))))
    for plans in ([p, p], [p, other], [p, f32], [p] * 9):
        ls, lg = ones(len(plans))
        with pytest.raises(krig.KrigError) as e:
            krig.mixture(plans, alpha, ls, lg)
        assert e.value.status == -1
