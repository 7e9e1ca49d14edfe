"""GPU: off-grid predictions (krig_interp) against the oracle's local Lagrange interpolation."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle.interp import interp_points
from oracle.rapid import Grid

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


def grid_of(w):
    return Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)


def points(g, n, seed):
    """Random points, plus the four corners, points on edges, and mesh nodes."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(0, g.m1 - 1, n)
    u = rng.uniform(0, g.m2 - 1, n)
    extra_t = [0, g.m1 - 1, 0, g.m1 - 1, 0, g.m1 - 1, 0.5, 3, 7]
    extra_u = [0, 0, g.m2 - 1, g.m2 - 1, 2.25, 1.5, 0, 5, g.m2 - 1]
    t = np.concatenate([t, extra_t])
    u = np.concatenate([u, extra_u])
    return np.stack([g.x0 + t * g.dx, g.y0 + u * g.dy], 1)


@pytest.fixture(scope="module")
def small(krig):
    w = wl.small_field()
    return w, {dt: krig.plan_for(w, dt) for dt in ("f64", "f32")}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("q", [2, 3, 4, 5, 6, 7, 8])
def test_interp_matches_oracle(krig, small, dtype, q):
    w, plans = small
    p = plans[dtype]
    g = grid_of(w)
    say("interp small field", dtype, "q", q)
    Y = np.random.default_rng(q).standard_normal((3, w.m1, w.m2))
    td = torch.float64 if dtype == "f64" else torch.float32
    yh = dev(Y, td)
    pts = points(g, 500, 10 + q)
    got = host(p.interp(yh, dev(pts), q))
    Yh = host(yh)  # the values the kernel read (rounded to FP32 in an FP32 plan)
    for b in range(3):
        ref = interp_points(g, Yh[b], pts, q)
        inside = ~np.isnan(ref)
        assert np.array_equal(np.isnan(got[b]), ~inside)
        scale = np.abs(Yh[b]).max()
        if dtype == "f64":
            # same polynomial, different rounding order of the Lagrange products
            assert np.abs(got[b][inside] - ref[inside]).max() < 1e-13 * scale
        else:  # FP64 arithmetic, one rounding of the output to FP32
            err = np.abs(got[b][inside] - ref[inside])
            assert np.all(err <= 2.0 ** -24 * np.abs(ref[inside]) + 1e-13 * scale)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_interp_nodes_exact_and_outside_nan(krig, small, dtype):
    w, plans = small
    p = plans[dtype]
    g = grid_of(w)
    say("interp nodes and outside points", dtype)
    td = torch.float64 if dtype == "f64" else torch.float32
    yh = dev(np.random.default_rng(5).standard_normal((2, w.m1, w.m2)), td)
    a = np.array([0, 1, 17, w.m1 - 1, 30, w.m1 - 2])
    b = np.array([0, w.m2 - 1, 40, w.m2 - 1, 0, 3])
    nodes = np.stack([g.x0 + a * g.dx, g.y0 + b * g.dy], 1)
    t = (nodes[:, 0] - g.x0) / g.dx
    u = (nodes[:, 1] - g.y0) / g.dy
    keep = (t == a) & (u == b)  # nodes whose FP64 coordinate maps back exactly
    assert keep.sum() >= 3
    Yh = host(yh)
    for q in (2, 4, 8):
        got = host(p.interp(yh, dev(nodes[keep]), q))
        assert np.array_equal(got, Yh[:, a[keep], b[keep]])
    outside = np.array([[g.x0 - 1e-3 * g.dx, g.y0], [g.x0, g.y0 + (g.m2 - 1) * g.dy * (1 + 1e-9) + 1e-9],
                        [np.nan, g.y0], [g.x0 + 1e6, g.y0 + 1e6]])
    assert np.all(np.isnan(host(p.interp(yh, dev(outside), 4))))


def test_interp_argument_errors_and_empty(krig, small):
    w, plans = small
    p = plans["f64"]
    say("interp argument errors")
    yh = dev(np.zeros((1, w.m1, w.m2)))
    pts = dev(np.zeros((3, 2)) + [[w.x0, w.y0]])
    for q in (0, 1, 9):
        with pytest.raises(krig.KrigError) as e:
            p.interp(yh, pts, q)
        assert e.value.status == -1
    out = p.interp(yh, dev(np.zeros((0, 2))), 4)
    assert tuple(out.shape) == (1, 0)
    assert p.lib.krig_interp(p.h, 1, yh.data_ptr(), 3, None, 4, None) == -1


def test_interp_full_size_sampled(krig):
    # the paper-sized mesh, 16 fields and a million points in the configuration the
    # bench times; sampled points checked one by one against the oracle
    w = wl.grad_batch(B=16)
    g = grid_of(w)
    say("interp full size 350x350, B=16, 1e6 points, q=4 f32")
    p = krig.plan_for(w, "f32")
    yhat = p.predict(dev(w.y))
    pts = points(g, 1_000_000, 99)
    got = p.interp(yhat, dev(pts), 4)
    again = p.interp(yhat, dev(pts), 4)
    G, A = host(got), host(again)
    assert np.array_equal(G, A)  # bitwise repeatable
    Yh = host(yhat)
    idx = np.concatenate([np.random.default_rng(1).choice(len(pts) - 9, 400, replace=False),
                          np.arange(len(pts) - 9, len(pts))])
    for b in (0, 7, 15):
        ref = interp_points(g, Yh[b], pts[idx], 4)
        err = np.abs(G[b, idx] - ref)
        assert np.all(err <= 2.0 ** -24 * np.abs(ref) + 1e-13 * np.abs(Yh[b]).max())
