"""GPU: krig_solve_noalloc, the solve for callers that cannot allocate device memory.

Through the C ABI: the allocation-free call must give krig_solve's result (same kernels,
same order: bit for bit) on two calls in a row, the second with a smaller input; leave the
device's free memory unchanged on a fresh plan; and reject a request beyond its scratch.
"""
import sys

import numpy as np
import pytest

import workloads as wl
from parity_bars import BAR_F64, check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_solve_noalloc_matches_solve(krig):
    big = wl.grad_batch(B=16)    # n = 1368, 16 fields
    small = wl.small_field()     # n = 200, then 3 fields
    pb, ps = krig.plan_for(big, "f64"), krig.plan_for(small, "f64")
    try:
        cases = [(pb, big.y, "paper field n=1368 B=16"),
                 (ps, np.stack([small.y[0], -small.y[0], 0.5 * small.y[0]]), "small field n=200 B=3")]
        for p, y, name in cases:  # two calls in a row, the second with a smaller input
            say("solve_noalloc", name)
            yd = dev(y)
            out = torch.empty(y.shape[0], p.n, dtype=torch.float64, device="cuda:0")
            got = host(p.solve_noalloc(yd, out))
            ref = host(p.solve(yd))
            check(f"solve_noalloc vs solve, {name}", relmax(got, ref), BAR_F64)
            assert np.array_equal(got, ref), name
        # the same inputs again after the smaller call: the shared scratch keeps no state
        out = torch.empty(16, pb.n, dtype=torch.float64, device="cuda:0")
        assert np.array_equal(host(pb.solve_noalloc(dev(big.y), out)), host(pb.solve(dev(big.y))))
    finally:
        pb.close()
        ps.close()


def test_solve_noalloc_allocates_nothing_and_checks_its_limit(krig):
    w = wl.paper_field()
    say("solve_noalloc on a fresh plan: free device memory, scratch limit")
    p = krig.plan_for(w, "f64")
    try:
        mb = p.info("SOLVE_NOALLOC_MAX_B")
        assert mb == 6132, mb  # B (n rounded up to 4) doubles <= 64 MiB
        y = dev(np.tile(w.y, (mb + 1, 1)))
        out = torch.empty(mb + 1, w.n, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        p.solve_noalloc(y[:mb], out[:mb])
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0  # the plan's workspaces were never grown
        with pytest.raises(krig.KrigError) as e:
            p.solve_noalloc(y, out)
        assert e.value.status == -1
        got = host(out[:mb])
        ref = host(p.solve(y[:mb]))  # krig_solve with the same B: the same tiles, the same bits
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[mb - 1], ref[mb - 1])
        one = host(p.solve(y[:1]))[0]  # B = 1 may take another tile form: equal to rounding
        assert np.abs(got[0] - one).max() <= 1e-12 * np.abs(one).max()
    finally:
        p.close()


def test_solve_in_place(krig):
    """krig_solve and krig_solve_noalloc with d_alpha == d_y (the header allows aliasing: y is
    read by the first triangular product, alpha written by the second): the in-place results
    must equal the out-of-place ones bit for bit, twice in a row."""
    w = wl.paper_field()
    say("in-place solves, paper field n=1368 B=16")
    p = krig.plan_for(w, "f64")
    try:
        ref = host(p.solve(dev(w.y)))
        for rep in range(2):
            y = dev(w.y)
            assert np.array_equal(host(p.solve(y, out=y)), ref), rep
            y = dev(w.y)
            assert np.array_equal(host(p.solve_noalloc(y, y)), ref), rep
    finally:
        p.close()
