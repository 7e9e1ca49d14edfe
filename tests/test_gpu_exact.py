"""GPU: exact kriging predictions (krig_predict_exact, krig_exact_at) against the oracle."""
import os
import sys

import numpy as np
import pytest

import workloads as wl
from oracle.exact import ExactKriging, gp_draw
from oracle.matern import Matern
from oracle.rapid import Grid

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS = np.finfo(np.float64).eps


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def check_bound(got, pts, sites, k, alpha, f32):
    """|got - exact| per point within the rounding bound of two n-term FP64 sums (each term
    carries a few eps from sqrt, the division and exp): 2 (n + 16) eps sum_i |k_ji alpha_i|,
    plus one FP32 rounding of the result for FP32 output."""
    K = k.cross(pts, sites)
    ref = alpha @ K.T
    S = np.abs(alpha) @ np.abs(K).T
    bound = 2 * (sites.shape[0] + 16) * EPS * S + (2.0 ** -24 * np.abs(ref) if f32 else 0.0)
    assert np.all(np.abs(got - ref) <= bound), float(np.max(np.abs(got - ref) / np.maximum(bound, 1e-300)))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_exact_grid_small_field(krig, dtype):
    w = wl.small_field()
    g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
    k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
    say("exact on the grid, small field", dtype)
    p = krig.plan_for(w, dtype)
    alpha = np.random.default_rng(3).standard_normal((3, w.n))
    got = host(p.exact(dev(alpha))).reshape(3, -1)
    check_bound(got, g.nodes(), w.sites, k, alpha, dtype == "f32")
    assert np.array_equal(host(p.exact(dev(alpha))).reshape(3, -1), got)  # bitwise repeatable


def test_exact_at_points_inside_and_outside(krig):
    w = wl.small_field()
    k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
    say("exact at points")
    p = krig.plan_for(w, "f32")
    rng = np.random.default_rng(4)
    pts = np.concatenate([rng.uniform(-0.3, 1.3, (700, 2)), w.sites[:5]])  # also outside, and on sites
    alpha = rng.standard_normal((2, w.n))
    got = host(p.exact_at(dev(alpha), dev(pts)))
    check_bound(got, pts, w.sites, k, alpha, False)
    assert host(p.exact_at(dev(alpha), dev(np.zeros((0, 2))))).shape == (2, 0)


def test_exact_paper_field_sampled(krig):
    # the paper-sized field with 16 fields on the full grid; sampled nodes against the oracle
    w = wl.grad_batch(B=16)
    g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
    k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
    say("exact on the paper field, B=16 f32")
    p = krig.plan_for(w, "f32")
    alpha = ExactKriging(w.sites, k).coef(w.y)
    got = host(p.exact(dev(alpha))).reshape(16, -1)
    idx = np.concatenate([np.random.default_rng(6).choice(g.m1 * g.m2, 1500, replace=False),
                          [0, g.m2 - 1, (g.m1 - 1) * g.m2, g.m1 * g.m2 - 1]])
    check_bound(got[:, idx], g.nodes()[idx], w.sites, k, alpha, True)


def test_rapid_equals_exact_when_sites_are_nodes(krig):
    # every site on a grid node: each weight vector is a unit vector, so the rapid
    # predictor is exact kriging (the closed special case of the method)
    m1, m2, L = 40, 36, 2
    dx, dy = 1.0 / (m1 - 1), 1.0 / (m2 - 1)
    rng = np.random.default_rng(7)
    q = rng.choice(m1 * m2, 60, replace=False)
    sites = np.stack([(q // m2) * dx, (q % m2) * dy], 1)
    say("rapid = exact with sites on nodes")
    p = krig.Plan(m1, m2, 0.0, 0.0, dx, dy, L, 1.0, 0.2, 1.5, 0.01, sites, "f64")
    alpha = dev(rng.standard_normal((2, 60)))
    rapid, exact = host(p.convolve(alpha)), host(p.exact(alpha))
    for b in range(2):
        assert np.abs(rapid[b] - exact[b]).max() <= 1e-12 * np.abs(exact[b]).max()


def test_exact_argument_errors(krig):
    w = wl.small_field()
    p = krig.plan_for(w, "f64")
    with pytest.raises(krig.KrigError) as e:
        p.exact(dev(np.zeros((0, w.n))))
    assert e.value.status == -1
    with pytest.raises(ValueError):
        p.exact_at(dev(np.zeros((1, w.n))), dev(np.zeros((3, 3))))


def test_factorial_cases_within_a_decade_of_table_a2(krig):
    # the accuracy study's measure through the GPU (rapid prediction against krig_exact_at at
    # five nodes from the centre to the corner, sigma2 = 1, exact data draws) for three factor
    # combinations, against the fitted log10 mean absolute error of Appendix A, Table A2
    coef = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "tableA2_coef.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                a_, b_ = line.split()
                coef[a_] = float(b_)
    r07 = {0.5: -np.log(0.7), 1.0: 0.7766915961392014, 1.5: 1.0973492107034915}  # phi(r07) = 0.7
    rng = np.random.default_rng(11)
    for nu, L, m, tau2, n, d07 in ((0.5, 2, 100, 0.01, 200, 0.4), (1.5, 4, 350, 0.1, 500, 0.2),
                                   (1.5, 2, 500, 0.5, 1500, 0.8), (1.0, 4, 100, 0.1, 500, 0.4)):
        model = coef["(Intercept)"]
        if nu != 0.5:
            sn = "smoothness1" if nu == 1.0 else "smoothness1.5"
            model += coef[sn] + (coef[f"{sn}:NN4"] if L == 4 else 0.0)
        model += coef["NN4"] if L == 4 else 0.0
        model += coef[f"nGrid{m}"] if m != 100 else 0.0
        model += coef[f"nugget{tau2}"] if tau2 != 0.01 else 0.0
        say("factorial case", nu, L, m, tau2, n, d07)
        k = Matern(1.0, d07 / r07[nu], nu, tau2)
        h = 1.0 / (m - 1)
        ab = [(m // 2, m // 2), (m // 4, m // 4), (0, 0), (m // 2, 0), (m - 1, m // 2)]
        idx = np.array([i * m + j for i, j in ab])
        pts = dev(np.array([[i * h, j * h] for i, j in ab]))
        errs = []
        for _ in range(3):
            s_ = rng.uniform(0, 1, (n, 2))
            p = krig.Plan(m, m, 0.0, 0.0, h, h, L, 1.0, k.rho, nu, tau2, s_, "f64")
            al = p.solve(dev(gp_draw(s_, k, rng)))
            rapid = host(p.convolve(al)).reshape(-1)[idx]
            errs.append(np.abs(rapid - host(p.exact_at(al, pts))[0]))
            p.close()
        got = np.log10(np.mean(errs))
        assert abs(got - model) < 1.0, (nu, L, m, tau2, got, model)


def test_kernel_at_matches_oracle(krig):
    # the interpolated covariance of a site (eq. weights) at off-grid points, with the
    # oracle's weights on both sides; M-term FP64 sums, bound as for the exact sum
    from oracle.rapid import RapidPredictor
    w = wl.small_field()
    g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
    k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
    rp = RapidPredictor(g, k, w.sites)
    say("kernel_at, small field")
    p = krig.plan_for(w, "f64")
    p.set_weights(dev(np.stack([rp.i0, rp.j0], 1), torch.int32), dev(rp.W))
    pts = np.random.default_rng(9).uniform(-0.1, 1.1, (500, 2))
    for i in (0, 17, w.n - 1):
        got = host(p.kernel_at(i, dev(pts)))
        ref = rp.approx_kernel(i, pts)
        S = w.sigma2 * np.abs(rp.W[i]).sum()  # bounds sum_m |W_im k_m|, as |k| <= sigma2
        assert np.all(np.abs(got - ref) <= 2 * (g.M + 16) * EPS * S), i
    with pytest.raises(krig.KrigError):
        p.kernel_at(w.n, dev(pts))


def test_table2_convergence_slopes_on_the_gpu(krig):
    # Figure 5 / Table 2 set-up through the GPU: range 0.25, L = 2, one site in the centre of
    # the central box, Lambda = sup over [0,1]^2 (a 121 x 121 lattice plus an 81 x 81 patch
    # around the site) of |k_approx - k|, against the inverse fill distance; slopes within
    # 0.2 of the paper's, for all four of its smoothness levels
    gold = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "table2_slopes.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                a_, b_ = line.split()
                gold[float(a_)] = float(b_)
    one = dev(np.ones((1, 1)))
    for nu in (0.5, 1.0, 1.5, 2.5):
        say("table 2 slopes on the GPU, nu", nu)
        errs, inv = [], []
        for m in (20, 30, 40, 60, 80, 100, 140):
            h = 1.0 / (m - 1)
            c = (m - 1) // 2
            s_ = np.array([[(c + 0.5) * h, (c + 0.5) * h]])
            p = krig.Plan(m, m, 0.0, 0.0, h, h, 2, 1.0, 0.25, nu, 0.0, s_, "f64")
            a = np.linspace(0, 1, 121)
            X, Y = np.meshgrid(a, a, indexing="ij")
            b = np.linspace(-3 * h, 3 * h, 81)
            U, V = np.meshgrid(b, b, indexing="ij")
            pts = dev(np.concatenate([np.stack([X.ravel(), Y.ravel()], 1), s_ + np.stack([U.ravel(), V.ravel()], 1)]))
            lam = (p.kernel_at(0, pts) - p.exact_at(one, pts)[0]).abs().max().item()
            errs.append(lam)
            inv.append(1.0 / (0.5 * np.hypot(h, h)))
            p.close()
        slope = -np.polyfit(np.log10(inv), np.log10(errs), 1)[0]
        assert abs(slope - gold[nu]) < 0.2, (nu, slope, gold[nu], errs)


def test_matern_nu1_values(krig):
    # nu = 1 has no elementary form: phi(r) = r K_1(r) by quadrature on the device, against
    # the oracle's Bessel evaluation over r from 1e-6 to 60 (exact_at with one unit coefficient)
    say("Matern nu = 1 values")
    k = Matern(1.7, 0.3, 1.0, 0.0)
    site = np.array([[0.5, 0.5]])
    p = krig.Plan(8, 8, 0.0, 0.0, 1 / 7, 1 / 7, 2, 1.7, 0.3, 1.0, 0.0, site, "f64")
    r = np.concatenate([[0.0], np.logspace(-6, np.log10(60.0), 400)])
    ang = np.random.default_rng(12).uniform(0, 2 * np.pi, r.size)
    pts = site + 0.3 * r[:, None] * np.stack([np.cos(ang), np.sin(ang)], 1)
    got = host(p.exact_at(dev(np.ones((1, 1))), dev(pts)))[0]
    ref = k.of_dist(np.hypot(pts[:, 0] - 0.5, pts[:, 1] - 0.5))
    assert np.all(np.abs(got - ref) <= 1e-14 * np.abs(ref) + 1e-300), float(np.max(np.abs(got - ref) / ref))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_predict_nu1_end_to_end(krig, dtype):
    # the whole predictor with nu = 1 (lag image, K_N, weights, solve, convolution) against
    # the oracle's direct form with its own weights
    from oracle.rapid import RapidPredictor, rapid_direct
    w = wl.tiny(seed=31, m1=40, m2=36, L=2, n=60, nu=1.0, rho=0.2, tau2=0.01, B=2)
    g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
    k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
    rp = RapidPredictor(g, k, w.sites)
    ek = ExactKriging(w.sites, k)
    say("predict nu = 1", dtype)
    p = krig.plan_for(w, dtype)
    got = host(p.predict(dev(w.y)))
    for b in range(2):
        ref = rapid_direct(g, k, rp.cstar(ek.coef(w.y[b]))).reshape(g.m1, g.m2)
        err = np.abs(got[b] - ref).max() / np.abs(ref).max()
        assert err < (1e-11 if dtype == "f64" else 1e-6), (b, err)
