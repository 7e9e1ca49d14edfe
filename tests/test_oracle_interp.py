"""Pins of the off-grid interpolation oracle (CPU only).

The interpolant is fixed by the mathematics of Lagrange interpolation: it reproduces
every polynomial of degree <= q-1 in each coordinate, takes the mesh value at a mesh
node, agrees with an independent library construction of the same polynomial, is
linear in the mesh values, and its error on a smooth function falls like h^q.
"""
import numpy as np
import pytest
from scipy.interpolate import lagrange

from oracle.interp import interp_points, lagrange_weights, stencil_start
from oracle.rapid import Grid


def grid(m1=17, m2=13):
    # dyadic origin and spacings: node coordinates and t = (x - x0)/dx are exact
    return Grid(m1, m2, -0.25, 1.125, 0.0625, 0.03125, 2)


def random_points(g, n, seed):
    rng = np.random.default_rng(seed)
    x = g.x0 + rng.uniform(0, g.m1 - 1, n) * g.dx
    y = g.y0 + rng.uniform(0, g.m2 - 1, n) * g.dy
    return np.stack([x, y], 1)


def mesh(g, f):
    X, Y = np.meshgrid(g.x0 + np.arange(g.m1) * g.dx, g.y0 + np.arange(g.m2) * g.dy, indexing="ij")
    return f(X, Y)


@pytest.mark.parametrize("q", [2, 3, 4, 6, 8])
def test_reproduces_tensor_polynomials(q):
    # every x^i y^j with i, j <= q-1 is reproduced exactly (up to rounding), also at the edges
    g = grid()
    pts = np.concatenate([random_points(g, 60, q),
                          [[g.x0, g.y0], [g.x0 + (g.m1 - 1) * g.dx, g.y0 + (g.m2 - 1) * g.dy]]])
    rng = np.random.default_rng(10 + q)
    coef = rng.standard_normal((q, q))

    def f(x, y):
        xs, ys = (x - 0.25) / 0.5, (y - 1.3) / 0.2
        return sum(coef[i, j] * xs ** i * ys ** j for i in range(q) for j in range(q))

    got = interp_points(g, mesh(g, f), pts, q)
    ref = f(pts[:, 0], pts[:, 1])
    assert np.max(np.abs(got - ref)) < 1e-10 * max(1.0, np.abs(ref).max())


def test_degree_q_is_not_reproduced():
    # a plain check that the pin above can fail: x^q is not reproduced by q nodes
    g = grid()
    pts = random_points(g, 40, 3)
    q = 3
    f = lambda x, y: ((x - 0.25) / 0.5) ** q
    assert np.max(np.abs(interp_points(g, mesh(g, f), pts, q) - f(pts[:, 0], pts[:, 1]))) > 1e-6


@pytest.mark.parametrize("q", [2, 4, 5])
def test_mesh_nodes_give_mesh_values(q):
    g = grid()
    Y = np.random.default_rng(1).standard_normal((g.m1, g.m2))
    a = np.array([0, 3, 7, g.m1 - 1, 5])
    b = np.array([0, 12, 4, g.m2 - 1, 0])
    pts = np.stack([g.x0 + a * g.dx, g.y0 + b * g.dy], 1)
    got = interp_points(g, Y, pts, q)
    assert np.allclose(got, Y[a, b], rtol=0, atol=1e-12)


@pytest.mark.parametrize("q", [2, 3, 4, 7])
def test_one_dimensional_case_matches_scipy_lagrange(q):
    # along a mesh row (u on a node) the interpolant is scipy's Lagrange polynomial
    # through the same q nodes, a construction independent of the product formula
    g = grid()
    Y = np.random.default_rng(2).standard_normal((g.m1, g.m2))
    b = 6
    for t in np.linspace(0.0, g.m1 - 1, 23):
        sx = stencil_start(t, g.m1, q)
        poly = lagrange(np.arange(sx, sx + q, dtype=float), Y[sx:sx + q, b])
        got = interp_points(g, Y, np.array([[g.x0 + t * g.dx, g.y0 + b * g.dy]]), q)[0]
        assert abs(got - poly(t)) < 1e-9 * max(1.0, np.abs(Y).max())


def test_stencil_rule():
    assert stencil_start(5.3, 17, 4) == 4          # i0 - 1 .. i0 + 2
    assert stencil_start(5.3, 17, 2) == 5          # the cell itself
    assert stencil_start(5.3, 17, 3) == 4          # i0 - 1 .. i0 + 1
    assert stencil_start(0.2, 17, 6) == 0          # shifted inward at the low edge
    assert stencil_start(16.0, 17, 4) == 13        # t = m - 1 sits in the last stencil
    assert stencil_start(15.9, 17, 8) == 9
    w = lagrange_weights(2.0, np.array([1.0, 2.0, 3.0]))
    assert np.array_equal(w, [0.0, 1.0, 0.0])
    assert np.isclose(lagrange_weights(0.37, np.arange(5.0)).sum(), 1.0)  # partition of unity


def test_linear_in_mesh_values_and_outside_is_nan():
    g = grid()
    rng = np.random.default_rng(4)
    Y1, Y2 = rng.standard_normal((2, g.m1, g.m2))
    pts = random_points(g, 30, 5)
    lhs = interp_points(g, 2.0 * Y1 - 3.0 * Y2, pts, 4)
    rhs = 2.0 * interp_points(g, Y1, pts, 4) - 3.0 * interp_points(g, Y2, pts, 4)
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-12)
    out = interp_points(g, Y1, np.array([[g.x0 - 1e-9, g.y0], [g.x0, g.y0 + (g.m2 - 1) * g.dy * 1.001]]), 4)
    assert np.all(np.isnan(out))


@pytest.mark.parametrize("q", [2, 4, 6])
def test_error_falls_like_h_to_the_q(q):
    # smooth field sampled on meshes of spacing h and h/2: the max error ratio is ~2^q
    f = lambda x, y: np.sin(2.1 * x + 0.3) * np.cos(1.7 * y - 0.2)
    errs = []
    for m in (41, 81):
        h = 1.0 / (m - 1)
        g = Grid(m, m, 0.0, 0.0, h, h, 1)
        pts = random_points(g, 200, 7)
        errs.append(np.max(np.abs(interp_points(g, mesh(g, f), pts, q) - f(pts[:, 0], pts[:, 1]))))
    rate = np.log2(errs[0] / errs[1])
    assert q - 0.6 < rate < q + 0.9, (errs, rate)
