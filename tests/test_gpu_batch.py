"""GPU: the uneven batch (krig_predict_many and the graph-recorded krig_batch).

Problems of different grids, site sets, kernels, neighbour orders and dtypes, drawn
like the 64-problem uneven workload at reduced n.  A batch must reproduce each plan's
own krig_predict bit for bit (same kernels, same inputs), on every replay of the
recorded graph, and each problem must match the FP64 oracle (with the oracle's
neighbour weights injected, so both sides start from identical inputs).  The full
64-problem workload (grids to 1024^2, n to 19,824) is compared with the oracle problem by
problem, in both dtypes, together with the FP64 solve of eq. findc at n >= 18,000.
"""
import sys

import numpy as np
import pytest

import workloads as wl
from parity_bars import bar_for, check
from oracle.exact import ExactKriging
from oracle.matern import Matern
from oracle.rapid import Grid, RapidPredictor, lag_quadrant, rapid_fft

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def relmax(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def problems(krig):
    """Eight uneven problems (n <= 2500), alternating FP32 / FP64 plans; problem 3
    has two fields and the last problem reuses plan 0 with other data."""
    ws = wl.uneven_batch(seed=4, count=7, nmax=2500)
    out = []
    for i, w in enumerate(ws):
        dtype = "f32" if i % 2 == 0 else "f64"
        say("uneven batch plan", i, w.name, dtype)
        g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
        k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
        rp = RapidPredictor(g, k, w.sites)
        ek = ExactKriging(w.sites, k)
        p = krig.plan_for(w, dtype)
        p.set_weights(dev(np.stack([rp.i0, rp.j0], 1), torch.int32), dev(rp.W))
        y = w.y if i != 3 else np.concatenate([w.y, -0.5 * w.y])
        out.append(dict(w=w, g=g, k=k, rp=rp, ek=ek, p=p, y=dev(y), dtype=dtype))
    last = dict(out[0])
    last["y"] = dev(0.25 * out[0]["w"].y[::-1].copy())
    out.append(last)
    return out


def reference(problems):
    return [host(q["p"].predict(q["y"])) for q in problems]


def test_problems_match_oracle(problems):
    for i, q in enumerate(problems[:-1]):
        say("uneven batch oracle", i, q["w"].name, q["dtype"])
        yhat = host(q["p"].predict(q["y"]))
        lag = lag_quadrant(q["g"], q["k"])
        for b in range(yhat.shape[0]):
            c = q["ek"].coef(host(q["y"])[b])
            cimg = q["rp"].cstar(c)
            ref = rapid_fft(q["g"], lag, cimg)
            cancel = np.abs(cimg).sum() / np.abs(ref).max()
            label = f"uneven (n <= 2500) problem {i} field {b}"
            check(f"{label} {q['dtype']}", relmax(yhat[b], ref), bar_for(q["dtype"], label),
                  f"cancellation {cancel:.3g}")


@pytest.mark.slow
def test_uneven_batch_full_size_against_oracle(krig):
    """Every problem of the 64-problem uneven workload at its full size, FP64 and FP32 plans,
    against the oracle's FFT form of eq. Convolution with the oracle's weights and
    coefficients (eq. findc by Cholesky) injected: the FP64 plan is held to 1e-12 (named
    exceptions only), the FP32 plan to 1e-5.  For n >= 18,000 the FP64 solve of eq. findc is
    compared with the oracle's Cholesky solve too: a backward-stable solve is within
    10 cond(M) eps, with cond(M) <= (n sigma2 + tau2) / tau2 (Gershgorin)."""
    ws = wl.uneven_batch(seed=4, count=64)
    failed = []

    def soft(label, err, bar, extra=""):
        try:
            check(label, err, bar, extra)
        except AssertionError as e:
            failed.append(e.args[0])

    for i, w in enumerate(ws):
        say("uneven full size", i, w.name)
        g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
        k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
        rp = RapidPredictor(g, k, w.sites)
        ek = ExactKriging(w.sites, k)
        alpha = ek.coef(w.y)
        del ek
        cimg = rp.cstar(alpha[0])
        ref = rapid_fft(g, lag_quadrant(g, k), cimg)
        cancel = np.abs(cimg).sum() / np.abs(ref).max()
        for dtype in ("f64", "f32"):
            p = krig.plan_for(w, dtype)
            try:
                if dtype == "f64" and w.n >= 18000:
                    bound = 10 * (w.n * w.sigma2 + w.tau2) / w.tau2 * np.finfo(float).eps
                    soft(f"uneven problem {i} solve n={w.n}", relmax(host(p.solve(dev(w.y)))[0], alpha[0]), bound)
                p.set_weights(dev(np.stack([rp.i0, rp.j0], 1), torch.int32), dev(rp.W))
                y = host(p.convolve(dev(alpha)))[0]
            finally:
                p.close()
            label = f"uneven problem {i}"
            soft(f"{label} ({w.name}) {dtype}", relmax(y, ref), bar_for(dtype, label), f"cancellation {cancel:.3g}")
    assert not failed, failed


def test_predict_many_bitwise(krig, problems):
    say("predict_many")
    ref = reference(problems)
    outs = [q["p"].empty(q["y"].shape[0], q["w"].m1, q["w"].m2) for q in problems]
    krig.predict_many([q["p"] for q in problems], [q["y"] for q in problems], outs)
    for i, (o, r) in enumerate(zip(outs, ref)):
        assert np.array_equal(host(o), r), i


@pytest.mark.parametrize("lanes", [1, 3])
def test_batch_graph_replays(krig, problems, lanes):
    say("batch graph, lanes", lanes)
    ref = reference(problems)
    outs = [q["p"].empty(q["y"].shape[0], q["w"].m1, q["w"].m2) for q in problems]
    bt = krig.Batch([q["p"] for q in problems], [q["y"] for q in problems], outs, lanes=lanes)
    try:
        for rep in range(3):
            for o in outs:
                o.fill_(float("nan"))  # a replay must write every output
            torch.cuda.synchronize()
            bt.launch()
            torch.cuda.synchronize()
            for i, (o, r) in enumerate(zip(outs, ref)):
                assert np.array_equal(host(o), r), (rep, i)
            # eager work on the same plans between replays
            host(problems[1]["p"].predict(problems[1]["y"]))
    finally:
        bt.close()


def test_batch_persistent_replays(krig, problems):
    """The work-queue (persistent) form, lanes = 0: every pass of all problems in one launch
    per pass and kernel form; each replay must reproduce every plan's own krig_predict bit for
    bit (problem 3 has two fields), with eager work on the plans between replays.  A plan
    that appears twice is refused (the problems run at once, each in its plan's workspaces)."""
    say("batch persistent form")
    qs = problems[:-1]  # distinct plans
    ref = reference(qs)
    outs = [q["p"].empty(q["y"].shape[0], q["w"].m1, q["w"].m2) for q in qs]
    bt = krig.Batch([q["p"] for q in qs], [q["y"] for q in qs], outs, lanes=0)
    try:
        for rep in range(3):
            for o in outs:
                o.fill_(float("nan"))  # a replay must write every output
            torch.cuda.synchronize()
            bt.launch()
            torch.cuda.synchronize()
            for i, (o, r) in enumerate(zip(outs, ref)):
                assert np.array_equal(host(o), r), (rep, i)
            host(qs[1]["p"].predict(qs[1]["y"]))
    finally:
        bt.close()
    with pytest.raises(krig.KrigError) as e:
        krig.Batch([problems[0]["p"], problems[-1]["p"]], [problems[0]["y"], problems[-1]["y"]], outs[:1] * 2, lanes=0)
    assert e.value.status == -1


def test_batch_persistent_paired_columns(krig):
    """Plans on the paired column form (F1 = 768 and 1024) in the persistent form reproduce
    their own krig_predict bit for bit (the queue walks the paired kernel's columns)."""
    ws = [wl.grad_batch(B=2), wl.tiny(seed=21, m1=450, m2=40, L=3, n=300, B=3, nu=1.5, rho=0.2, tau2=0.05)]
    plans, ys, outs = [], [], []
    for w, v in zip(ws, (3, 5)):
        p = krig.plan_for(w, "f64")
        p.tune("COLS_PAIR", v)
        plans.append(p)
        ys.append(dev(w.y))
        outs.append(p.empty(w.y.shape[0], w.m1, w.m2))
    say("batch persistent form, paired columns", [p.F1 for p in plans])
    ref = reference([dict(p=p, y=y) for p, y in zip(plans, ys)])
    bt = krig.Batch(plans, ys, outs, lanes=0)
    try:
        for rep in range(2):
            for o in outs:
                o.fill_(float("nan"))
            torch.cuda.synchronize()
            bt.launch()
            torch.cuda.synchronize()
            for i, (o, r) in enumerate(zip(outs, ref)):
                assert np.array_equal(host(o), r), (rep, i)
    finally:
        bt.close()
        for p in plans:
            p.close()


@pytest.mark.parametrize("lanes", [0, 2])
def test_batch_tile_forms(krig, lanes):
    """Problems whose solves take each tile form of the triangular products (8 x 8: n = 700 with
    16 fields; 16 x 16: n = 2100 with 17 and n = 700 with 64; 64 x 64 blocks: n = 4100 with 260
    fields, which the persistent form launches per problem) reproduce their own krig_predict bit
    for bit in the persistent form and over graph branches.  The site sets are dense enough for
    the scatter's own kernel (1.3 to 7.8 CSR entries per padded node); the first problem is set
    to the fused scatter, so both scatter forms share the batch."""
    rng = np.random.default_rng(17)
    shapes = [(700, 16), (2100, 17), (700, 64), (4100, 260)]
    plans, ys, outs = [], [], []
    try:
        for i, (n, B) in enumerate(shapes):
            sites = rng.uniform(0.0, 1.0, (n, 2))
            p = krig.Plan(96, 80, 0.0, 0.0, 1 / 95, 1 / 79, 2, 1.0, 0.15, 1.5, 0.05, sites,
                          "f64" if i % 2 else "f32")
            plans.append(p)
            ys.append(dev(rng.standard_normal((B, n))))
            outs.append(p.empty(B, 96, 80))
        assert all(p.info("SCATTER") == 2 for p in plans)
        plans[0].tune("SCATTER", 1)
        say("batch tile forms, lanes", lanes, shapes)
        ref = reference([dict(p=p, y=y) for p, y in zip(plans, ys)])
        bt = krig.Batch(plans, ys, outs, lanes=lanes)
        try:
            for rep in range(2):
                for o in outs:
                    o.fill_(float("nan"))
                torch.cuda.synchronize()
                bt.launch()
                torch.cuda.synchronize()
                for i, (o, r) in enumerate(zip(outs, ref)):
                    assert np.array_equal(host(o), r), (rep, i)
        finally:
            bt.close()
    finally:
        for p in plans:
            p.close()


def test_batch_guards(krig, problems):
    """While a batch exists its plans refuse destruction and workspace growth."""
    say("batch guards")
    q = problems[2]
    p = q["p"]
    outs = [p.empty(1, q["w"].m1, q["w"].m2)]
    bt = krig.Batch([p], [q["y"]], outs, lanes=1)
    try:
        big = torch.zeros(64, p.n, dtype=torch.float64, device="cuda:0")
        with pytest.raises(krig.KrigError) as e:
            p.predict(big)
        assert e.value.status == -1
        assert p.lib.krig_plan_destroy(p.h) == -1
        p.timing(True)
        try:
            with pytest.raises(krig.KrigError) as e:
                krig.Batch([p], [q["y"]], outs, lanes=1)
            assert e.value.status == -1
        finally:
            p.timing(False)
    finally:
        bt.close()
    host(p.predict(torch.zeros(64, p.n, dtype=torch.float64, device="cuda:0")))  # grows now


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_step_graph_replays(krig, dtype):
    """predict + adjoint recorded once in a HIP graph (torch capture of the plan's
    calls: sized workspaces, no host synchronisation or memset inside) and replayed:
    every replay must reproduce the eager step bit for bit, with eager work on the
    same plan between the replays."""
    w = wl.grad_batch(B=4)
    say("step graph replays", dtype)
    p = krig.plan_for(w, dtype)
    y = dev(w.y)
    B = y.shape[0]
    alpha = torch.empty(B, w.n, dtype=torch.float64, device="cuda:0")
    saved = p.new_saved(B)
    yhat = p.empty(B, w.m1, w.m2)
    dy = torch.empty(B, w.n, dtype=torch.float64, device="cuda:0")
    dlag = p.empty(w.m1 + w.L, w.m2 + w.L)
    g = (2.0 * dev(w.extra["mask"], yhat.dtype) * p.predict(y)).contiguous()

    def step():
        p.predict(y, alpha_out=alpha, saved=saved, out=yhat)
        p.adjoint(g, alpha=alpha, saved=saved, dy_out=dy, dlag_out=dlag)

    step()
    ref = [host(t) for t in (alpha, yhat, dy, dlag)]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        for t in (alpha, yhat, dy, dlag):
            t.fill_(float("nan"))  # a replay must write every output
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for name, t, r in zip(("alpha", "yhat", "dy", "dlag"), (alpha, yhat, dy, dlag), ref):
            assert np.array_equal(host(t), r), (rep, name)
        host(p.predict(y))  # eager work on the same plan between replays
    del graph
