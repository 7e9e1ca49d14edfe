"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only)."""
import os

import numpy as np
import pytest
from scipy import special

from oracle import philox
from oracle.exact import ExactKriging, gp_draw
from oracle.matern import Matern, phi, phi_closed, phi_general
from oracle.rapid import (Grid, RapidPredictor, conv_lag_direct, cstar_image, embed_even, fft_len,
                          filter_spectrum_centered, filter_spectrum_reflected, grid_unit, kn_matrix, kvecs,
                          lag_quadrant, neighbour_weights, offsets, rapid_direct, rapid_fft, rapid_fft_spectrum,
                          site_cells, sparse_A)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------- Matern (eq. Matern1)
@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_closed_forms_match_bessel_definition(nu):
    r = np.geomspace(1e-3, 30.0, 400)
    a = phi_closed(r, nu)
    b = phi_general(r, nu)
    assert np.max(np.abs(a - b) / np.abs(b)) < 1e-13


def test_phi_at_zero_and_half_integer_identity():
    # phi(0) = 1 for every nu (limit of d^nu K_nu(d) normalised); nu = 1/2 is exp(-d)
    for nu in (0.5, 1.0, 1.5, 2.5):
        assert phi(np.array([0.0]), nu)[0] == 1.0
        assert abs(phi_general(np.array([1e-9]), nu)[0] - 1.0) < 1e-6
    d = np.linspace(0.01, 5, 50)
    assert np.allclose(phi(d, 0.5), np.exp(-d), rtol=1e-15)
    # K_{1/2}(d) = sqrt(pi / (2 d)) e^{-d}, a textbook identity independent of scipy's kv
    assert np.allclose(special.kv(0.5, d), np.sqrt(np.pi / (2 * d)) * np.exp(-d), rtol=1e-13)


def test_range_divides_distance():
    k = Matern(2.0, 0.3, 1.5)
    assert np.isclose(k.of_dist(0.3), 2.0 * phi(np.array([1.0]), 1.5)[0])
    # doubling range == halving distance (the paper's equivalence remark in Section 3.2)
    k2 = Matern(2.0, 0.6, 1.5)
    assert np.allclose(k2.of_dist(np.array([0.2, 0.5])), k.of_dist(np.array([0.1, 0.25])))


# ---------------------------------------------------------------------- K_N (Step 1)
def test_kn_structure():
    g = Grid(30, 40, 0.0, 0.0, 2.0 / 29, 1.0 / 39, 3)
    k = Matern(1.3, 0.3, 2.5)
    KN = kn_matrix(g, k)
    assert KN.shape == (36, 36)
    assert np.array_equal(KN, KN.T)
    assert np.all(np.diag(KN) == 1.3)
    off = offsets(3)
    # block-Toeplitz: entries depend only on the offset difference
    for p in range(36):
        for q in range(36):
            d = tuple(off[p] - off[q])
            hx, hy = d[0] * g.dx, d[1] * g.dy
            assert KN[p, q] == k.of_lag(hx, hy)
    # lexicographic ox-major order
    assert tuple(off[0]) == (-2, -2) and tuple(off[1]) == (-2, -1) and tuple(off[6]) == (-1, -2)


def test_site_cells_floor_and_domain():
    g = grid_unit(11, 11, 2)
    s = np.array([[0.0, 0.0], [1.0, 1.0], [0.1, 0.35], [0.55, 0.999]])
    i0, j0, u, v = site_cells(g, s)
    assert list(i0) == [0, 10, 1, 5] and list(j0) == [0, 10, 3, 9]
    assert np.all((u >= 0) & (u < 1)) and np.all((v >= 0) & (v < 1))
    with pytest.raises(ValueError):
        site_cells(g, np.array([[1.0 + 1e-9, 0.5]]))
    with pytest.raises(ValueError):
        site_cells(g, np.array([[0.5, -1e-12]]))


# ---------------------------------------------------------------------- weights (eq. weights)
def _tiny_geom(L=2, nu=1.5):
    g = Grid(12, 14, 0.1, -0.2, 0.09, 0.07, L)
    k = Matern(1.0, 0.35, nu)
    return g, k


@pytest.mark.parametrize("L", [1, 2, 3])
def test_weights_satisfy_interpolation_condition(L):
    g, k = _tiny_geom(L)
    rng = np.random.default_rng(1)
    s = np.stack([g.x0 + rng.uniform(0, (g.m1 - 1) * g.dx, 40), g.y0 + rng.uniform(0, (g.m2 - 1) * g.dy, 40)], 1)
    i0, j0, W = neighbour_weights(g, k, s)
    _, _, u, v = site_cells(g, s)
    KN = kn_matrix(g, k)
    kv = kvecs(g, k, u, v)
    cond = np.linalg.cond(KN)
    res = np.abs(W @ KN - kv).max()
    assert res < 1e3 * np.finfo(float).eps * max(1.0, np.abs(W).max() * np.abs(KN).max()) * g.M
    # and k_i really is the covariance of the site with its neighbours (recomputed from coordinates)
    off = offsets(L)
    for i in range(5):
        nx = g.x0 + (i0[i] + off[:, 0]) * g.dx
        ny = g.y0 + (j0[i] + off[:, 1]) * g.dy
        kk = k.cross(s[i:i + 1], np.stack([nx, ny], 1))[0]
        assert np.allclose(kk, kv[i], rtol=1e-12, atol=1e-15)
    assert cond > 1  # sanity


def test_site_on_node_gets_unit_weight_vector():
    g, k = _tiny_geom(2)
    # node (4, 6) exactly: t integer -> anchor is that node, offset (0, 0)
    s = np.array([[g.x0 + 4 * g.dx, g.y0 + 6 * g.dy]])
    i0, j0, u, v = site_cells(g, s)
    # the FP64 division may land just below the integer; accept either cell but require
    # the weight to be a unit vector on the node itself
    i0, j0, W = neighbour_weights(g, k, s)
    off = offsets(2)
    q = np.where((i0[0] + off[:, 0] == 4) & (j0[0] + off[:, 1] == 6))[0]
    assert len(q) == 1
    e = np.zeros(g.M)
    e[q[0]] = 1.0
    cond = np.linalg.cond(kn_matrix(g, k))
    assert np.abs(W[0] - e).max() < 1e3 * np.finfo(float).eps * cond


def test_weights_mirror_symmetry():
    # reflecting the site about the centre of its cell reflects the weights
    g = Grid(10, 10, 0.0, 0.0, 0.1, 0.1, 2)
    k = Matern(1.0, 0.3, 1.5)
    s = np.array([[0.4 + 0.1 * 0.3, 0.5 + 0.1 * 0.6], [0.4 + 0.1 * 0.7, 0.5 + 0.1 * 0.6]])
    _, _, W = neighbour_weights(g, k, s)
    off = offsets(2)
    # offset ox -> 1 - ox maps the neighbourhood of u onto that of 1 - u
    perm = [int(np.where((off[:, 0] == 1 - ox) & (off[:, 1] == oy))[0][0]) for ox, oy in off]
    cond = np.linalg.cond(kn_matrix(g, k))
    assert np.abs(W[1] - W[0][perm]).max() < 1e4 * np.finfo(float).eps * cond
    # transpose symmetry when dx == dy: swapping (u, v) swaps (ox, oy)
    s2 = np.array([[0.4 + 0.1 * 0.6, 0.5 + 0.1 * 0.3]])
    _, _, W2 = neighbour_weights(g, k, s2)
    perm2 = [int(np.where((off[:, 0] == oy) & (off[:, 1] == ox))[0][0]) for ox, oy in off]
    s3 = np.array([[0.4 + 0.1 * 0.3, 0.5 + 0.1 * 0.6]])
    _, _, W3 = neighbour_weights(g, k, s3)
    assert np.abs(W2[0] - W3[0][perm2]).max() < 1e4 * np.finfo(float).eps * cond


# ---------------------------------------------------------------------- Steps 5-7
def _tiny_problem(seed=0, m1=9, m2=11, L=2, n=13):
    rng = np.random.default_rng(seed)
    g = Grid(m1, m2, 0.0, 0.0, 1.0 / (m1 - 1), 1.3 / (m2 - 1), L)
    k = Matern(1.0, 0.4, 1.5)
    s = np.stack([rng.uniform(0, 1.0, n), rng.uniform(0, 1.3, n)], 1)
    return g, k, s, rng


def test_scatter_matches_dense_brute_force():
    g, k, s, rng = _tiny_problem()
    rp = RapidPredictor(g, k, s)
    c = rng.standard_normal(len(s))
    # dense A built entry by entry from the definition
    A = np.zeros((len(s), g.P1 * g.P2))
    off = offsets(g.L)
    for i in range(len(s)):
        for m, (ox, oy) in enumerate(off):
            p, q = rp.i0[i] + g.L + ox, rp.j0[i] + g.L + oy
            A[i, p * g.P2 + q] += rp.W[i, m]
    img = rp.cstar(c)
    assert np.abs(img.ravel() - A.T @ c).max() < 1e-14 * np.abs(A.T @ c).max()
    # mass: sum of c* = sum_i c_i sum_m W_im
    assert np.isclose(img.sum(), np.sum(c * rp.W.sum(1)), rtol=1e-13)
    # support stays inside the padded grid's interior ring
    nz = np.nonzero(img)
    assert nz[0].min() >= 1 and nz[1].min() >= 1


def test_direct_convolution_matches_brute_force_and_delta():
    g, k, s, rng = _tiny_problem(1)
    cimg = np.zeros((g.P1, g.P2))
    cimg[3, 5] = 1.0
    y = rapid_direct(g, k, cimg).reshape(g.m1, g.m2)
    # delta at padded (3, 5): output (a, b) = k(s_(a,b) - s_(3-L, 5-L))
    a, b = np.meshgrid(np.arange(g.m1), np.arange(g.m2), indexing="ij")
    ref = k.of_lag((a + g.L - 3) * g.dx, (b + g.L - 5) * g.dy)
    assert np.abs(y - ref).max() < 1e-15
    # random image: direct sum vs the lag-table form vs the FFT variant
    cimg = rng.standard_normal((g.P1, g.P2))
    y1 = rapid_direct(g, k, cimg).reshape(g.m1, g.m2)
    lag = lag_quadrant(g, k)
    y2 = conv_lag_direct(g, lag, cimg)
    y3 = rapid_fft(g, lag, cimg)
    sc = np.abs(y1).max()
    assert np.abs(y1 - y2).max() < 1e-13 * sc
    assert np.abs(y1 - y3).max() < 1e-13 * sc


def test_reflection_free_filter_setup():
    """The remark after Step 7: the filter spectrum from the covariance about the torus centre
    and one extra FFT (the centre indicator's) instead of reflecting the lag quadrant."""
    g, k, s, rng = _tiny_problem(2)
    F1, F2 = fft_len(g.m1 + g.P1 - 1), fft_len(g.m2 + g.P2 - 1)
    cen = filter_spectrum_centered(g, k, F1, F2)
    # the centred image is even about the centre, so after the phase is divided out the
    # spectrum is real
    assert np.abs(cen.imag).max() < 1e-13 * np.abs(cen.real).max()
    # it is the spectrum of the full minimal-image lag table (every lag up to half the torus)
    full = k.of_lag(np.arange(F1 // 2 + 1)[:, None] * g.dx, np.arange(F2 // 2 + 1)[None, :] * g.dy)
    ref = np.fft.fft2(embed_even(full, F1, F2)).real
    assert np.abs(cen.real - ref).max() < 1e-13 * np.abs(ref).max()
    # it differs from the reflected quadrant's spectrum (middle lags filled), yet the kept
    # outputs are the direct sum's, as the reflected filter's are
    refl = filter_spectrum_reflected(lag_quadrant(g, k), F1, F2)
    assert np.abs(cen.real - refl).max() > 1e-6 * np.abs(refl).max()
    cimg = rng.standard_normal((g.P1, g.P2))
    y0 = rapid_direct(g, k, cimg).reshape(g.m1, g.m2)
    sc = np.abs(y0).max()
    assert np.abs(rapid_fft_spectrum(g, cen.real, cimg) - y0).max() < 1e-13 * sc
    assert np.abs(rapid_fft_spectrum(g, refl, cimg) - y0).max() < 1e-13 * sc
    # a delta at padded (3, 5) gives the shifted covariance through the centred filter too
    d = np.zeros((g.P1, g.P2))
    d[3, 5] = 1.0
    a, b = np.meshgrid(np.arange(g.m1), np.arange(g.m2), indexing="ij")
    assert np.abs(rapid_fft_spectrum(g, cen.real, d) - k.of_lag((a + g.L - 3) * g.dx, (b + g.L - 5) * g.dy)).max() < 1e-14


def test_fft_len_and_embedding():
    assert fft_len(2 * 350 + 6 - 1) == 768
    assert fft_len(2 * 512 + 8 - 1) == 1152
    assert fft_len(2 * 64 + 4 - 1) == 144
    lag = np.arange(12.0).reshape(3, 4)
    E = embed_even(lag, 8, 10)
    assert E[0, 0] == 0 and E[1, 2] == lag[1, 2] and E[7, 8] == lag[1, 2] and E[2, 3] == lag[2, 3]
    assert E[4, 0] == 0.0  # lag 4 outside the quadrant -> zero
    assert np.array_equal(E, E[np.r_[0, 7:0:-1]][:, np.r_[0, 9:0:-1]])  # even


def test_sites_on_nodes_make_rapid_equal_exact():
    # A rows are unit vectors, so k_approx(., s_i) = k(., s_i) exactly (eq. ApproxCovariance)
    g = grid_unit(24, 20, 2)
    k = Matern(1.0, 0.2, 1.5, 1e-3)
    rng = np.random.default_rng(5)
    ia = rng.integers(2, 21, 30)
    ib = rng.integers(2, 17, 30)
    s = np.stack([g.x0 + ia * g.dx, g.y0 + ib * g.dy], 1)
    s = np.unique(s, axis=0)
    ek = ExactKriging(s, k)
    y = rng.standard_normal(len(s))
    c = ek.coef(y)
    rp = RapidPredictor(g, k, s)
    yr = rp.predict_direct(c)
    ye = ek.predict_at(g.nodes(), c)
    assert np.abs(yr - ye).max() < 1e-12 * np.abs(ye).max()


def test_exact_kriging_interpolates_without_nugget():
    g = grid_unit(15, 15, 2)
    k = Matern(1.0, 0.2, 1.5, 0.0)
    rng = np.random.default_rng(2)
    idx = rng.choice(15 * 15, 20, replace=False)
    s = g.nodes()[idx]
    ek = ExactKriging(s, k)
    y = rng.standard_normal(20)
    yhat = ek.predict_at(s, ek.coef(y))
    assert np.abs(yhat - y).max() < 1e-9


def test_linearity_in_data():
    g, k, s, rng = _tiny_problem(3)
    k = Matern(1.0, 0.4, 1.5, 1e-2)
    ek = ExactKriging(s, k)
    rp = RapidPredictor(g, k, s)
    y1, y2 = rng.standard_normal((2, len(s)))
    f = lambda y: rp.predict_direct(ek.coef(y))
    lhs = f(2.0 * y1 - 3.0 * y2)
    rhs = 2.0 * f(y1) - 3.0 * f(y2)
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


def test_approximation_error_falls_with_L_smoothness_and_resolution():
    rng = np.random.default_rng(11)
    s = rng.uniform(0.05, 0.95, (60, 2))

    def err(m, L, nu):
        g = grid_unit(m, m, L)
        k = Matern(1.0, 0.25, nu, 0.01)
        ek = ExactKriging(s, k)
        c = ek.coef(np.sin(3 * s[:, 0]) + np.cos(2 * s[:, 1]))
        rp = RapidPredictor(g, k, s)
        idx = np.arange(0, m * m, 7)
        return np.abs(rp.predict_direct(c, idx) - ek.predict_at(g.nodes()[idx], c)).mean()

    assert err(40, 3, 1.5) < 0.5 * err(40, 2, 1.5)      # larger L
    assert err(40, 2, 2.5) < 0.5 * err(40, 2, 0.5)      # smoother kernel
    assert err(80, 2, 1.5) < 0.5 * err(40, 2, 1.5)      # finer grid


def test_expected_error_is_zero_over_data_draws():
    # E[g_approx - g_hat] = 0 under the model (Section 3, after eq. error1)
    g = grid_unit(20, 20, 2)
    k = Matern(1.0, 0.3, 1.5, 0.05)
    rng = np.random.default_rng(4)
    s = rng.uniform(0, 1, (40, 2))
    ek = ExactKriging(s, k)
    rp = RapidPredictor(g, k, s)
    idx = np.array([0, 210, 399])
    errs = []
    for _ in range(300):
        c = ek.coef(gp_draw(s, k, rng))
        errs.append(rp.predict_direct(c, idx) - ek.predict_at(g.nodes()[idx], c))
    errs = np.array(errs)
    se = errs.std(0) / np.sqrt(len(errs))
    assert np.all(np.abs(errs.mean(0)) < 4 * se)


# ---------------------------------------------------------------------- Philox
def test_philox_known_answers():
    for line in open(os.path.join(GOLD, "philox_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        out = philox.philox4x32(w[0:4], w[4:6])
        assert [int(x) for x in out] == w[6:10]


def test_box_muller_moments():
    e = np.arange(200000, dtype=np.uint64)
    w = philox.philox4x32((e, 7, 0, 0), philox.split_seed(123))
    a, b = philox.box_muller(w[0], w[1])
    for z in (a, b):
        assert abs(z.mean()) < 0.01 and abs(z.var() - 1) < 0.01
    assert abs(np.mean(a * b)) < 0.01
