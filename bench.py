"""Benchmark: grid predictions/s of the rapid Kriging predictor, forward + adjoint, on one GPU.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Workload (one step): the paper-sized field -- n = 1368 sites on [0,2] x [0,1],
Matern nu = 2.5, range 0.3, nugget 0.05, 350 x 350 grid, L = 3 -- with a batch
of B = 16 data vectors: y -> alpha (FP64 solve) -> scatter + FFT convolution ->
y_hat, then the adjoint of an upstream gradient g = 2 m y_hat (loss sum m y_hat^2,
m a seeded U[0,1] mask) -> dy (FP64 solve) and d lag.  Inputs are resident in
HBM before timing.  The timed steps are the call loop; the same step recorded once
as a HIP graph and replayed is timed too (graph_ms_per_step; --graph makes it the
timed figure).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
PROFILES = os.path.join(ROOT, "profiles")
# sources of the FFT pass kernels: a recorded traffic figure holds only while they are unchanged
KERNEL_SOURCES = ["fft_passes.h", "fft_args.h", "fft_reg.h", "krig_internal.h", "matern_dev.h", "philox_dev.h",
                  "spec_io.h", "fft_body_rows_r2c.inc", "fft_body_cols.inc", "fft_body_rows_c2r.inc"]
STAGE_SOURCES = {"INTERP": ["interp.hip", "interp.h"]}  # stages whose kernel lives elsewhere


def kernel_source_hash(stage=None):
    h = hashlib.sha256()
    for name in STAGE_SOURCES.get(stage, KERNEL_SOURCES):
        with open(os.path.join(ROOT, "paper_2605_29284_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(stage):
    """HBM bytes per launch of a stage's kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is none or
    the kernel sources have changed since it was taken."""
    if not os.path.isdir(PROFILES):
        return None
    for name in sorted(os.listdir(PROFILES)):
        if not name.startswith(stage + "_") or not name.endswith(".md"):
            continue
        txt = open(os.path.join(PROFILES, name)).read()
        m = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)\s*$", txt, re.M)
        h = re.search(r"^kernel_source_hash:\s*([0-9a-f]+)\s*$", txt, re.M)
        if m and h and h.group(1) == kernel_source_hash(stage):
            return float(m.group(1))
    return None


def stage_bytes(p, B, model="s8d"):
    """Algorithmic bytes per launch of each timed single-kernel stage of the grad-batch step (B
    fields), in one of two models:
      "s8d"  the survey's measurement model: 8-byte complex spectra and 4-byte caller arrays
             (FP32), the filter spectrum in FP32, CSR entries of 8 bytes; the adjoint's column
             pass reads G-hat (m1 rows), writes the correlation spectra (P1 rows) and reloads the
             saved spectrum of c* as a full F1 x H2 spectrum per field, and writes the summed
             lag-gradient spectrum once; the padded correlation image is FP32;
      "build" what this build's kernels must move: FP64 spectra between the passes (FP32 for the
             prediction's column-pass output in FP32 plans), the filter in FP64, the plan's dtype
             for caller arrays, an FP64 correlation image.
    Per-group partial lag-gradient spectra are an implementation choice and count once."""
    m1, m2, n, M = p.m1, p.m2, p.n, p.M
    P1, P2, F1, H2 = p.P1, p.P2, p.F1, p.info("H2")
    if model == "s8d":
        z = zs = zg = zp = 8
        t, fb, img, ent = 4, 4, 4, 8
        adj_c = F1
    else:
        f32 = p.dtype_code == 1
        z, zs, zg, zp = 16, (8 if f32 else 16), 16, 16
        t, fb, img, ent = (4 if f32 else 8), 8, 8, 12
        adj_c = P1
    return {
        "ROWS_FWD": B * (n * 8 + H2 * P1 * z) + n * M * ent + (P1 * P2 + 1) * 4,
        "COLS_CONV": B * (H2 * P1 * z + H2 * m1 * zs) + H2 * F1 * fb,
        "ROWS_INV": B * (H2 * m1 * zs + m1 * m2 * t),
        "ADJ_ROWS_FWD": B * (m1 * m2 * t + H2 * m1 * zg),
        "ADJ_COLS": B * (H2 * m1 * zg + H2 * P1 * z + H2 * adj_c * z) + H2 * F1 * fb + H2 * F1 * zp,
        "ADJ_ROWS_INV": B * (H2 * P1 * z + P1 * P2 * img),
        "GATHER": B * (P1 * P2 * img + n * 8) + n * M * 8,
    }


def cpu_baseline(w, nfields: int, reps: int = 6):
    """The FP64 oracle (its FFT variants, single thread) on a bounded sample of fields; also
    returns the oracle's weights and its outputs for fields 0 .. nfields-1 (y_hat, dy and the
    summed d lag, with the upstream gradient g = 2 m y_hat rounded to FP32 so that both plans
    can take the same g), for the error report."""
    from threadpoolctl import threadpool_limits

    from oracle.exact import ExactKriging
    from oracle.grad import corr_image_fft, dlag_fft, grad_coef
    from oracle.matern import Matern
    from oracle.rapid import Grid, RapidPredictor, lag_quadrant, rapid_fft

    outs = {"yhat": [], "dy": [], "g": [], "dlag": 0.0}
    with threadpool_limits(limits=1):
        g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
        k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
        ek = ExactKriging(w.sites, k)
        rp = RapidPredictor(g, k, w.sites)
        lag = lag_quadrant(g, k)
        mask = w.extra["mask"]
        t0 = time.perf_counter()
        for it, b in enumerate([f % w.B for f in range(nfields * reps)]):
            c = ek.coef(w.y[b])
            cimg = rp.cstar(c)
            yhat = rapid_fft(g, lag, cimg)
            gup = (2.0 * mask * yhat).astype(np.float32).astype(np.float64)
            dy = ek.coef(grad_coef(rp.A, corr_image_fft(g, lag, gup)))
            dl = dlag_fft(g, gup, cimg)
            if it < nfields:
                outs["yhat"].append(yhat)
                outs["dy"].append(dy)
                outs["g"].append(gup)
                outs["dlag"] = outs["dlag"] + dl
        dt = time.perf_counter() - t0
    res = {"value": nfields * reps * w.m1 * w.m2 / dt, "unit": "grid predictions/s", "cores": 1, "kind": "oracle",
           "sample": f"{nfields} of the {w.B} fields x {reps} passes, forward + adjoint (y -> y_hat, g -> dy, d lag) with "
                     f"the oracle's FP64 FFT variants, one thread, {dt:.1f} s", "host": host_cpu()}
    return res, dict(anchor=np.stack([rp.i0, rp.j0], 1), W=rp.W, **outs)


def oracle_errors(torch, krig, w, p, ref, dev):
    """Relative max errors of one plan against the oracle on identical inputs: the oracle's
    weights injected (the plan is changed: call after its timings), the same data vectors and
    the same FP32-rounded upstream gradients.  y_hat per field (max over fields), dy over the
    fields, d lag summed over them."""
    nf = len(ref["yhat"])
    p.set_weights(torch.as_tensor(ref["anchor"], dtype=torch.int32, device=dev),
                  torch.as_tensor(ref["W"], dtype=torch.float64, device=dev))
    y = torch.as_tensor(w.y[:nf], dtype=torch.float64, device=dev)
    alpha = torch.empty(nf, w.n, dtype=torch.float64, device=dev)
    saved = p.new_saved(nf)
    yh = p.predict(y, alpha_out=alpha, saved=saved).double().cpu().numpy()
    gup = torch.as_tensor(np.stack(ref["g"]), dtype=p.tdtype, device=dev)
    dy, dlag = p.adjoint(gup, alpha=alpha, saved=saved)
    dy, dlag = dy.cpu().numpy(), dlag.double().cpu().numpy()
    rel = lambda a, b: float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    return {"yhat": max(rel(yh[b], ref["yhat"][b]) for b in range(nf)), "dy": rel(dy, np.stack(ref["dy"])),
            "dlag": rel(dlag, ref["dlag"])}


def host_cpu():
    """Model name and logical CPU count of the host that timed the oracle."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def uneven(a, torch, krig, wl, dev):
    """The 64-problem uneven batch (grids 128^2..1024^2, n 500..20000, L 2..4, nu 0.5..2.5),
    recorded once as a HIP graph and replayed; FP32 plans against FP64 plans, one dtype at a
    time (their inverse factors take tens of GB).  Prints one JSON line."""
    ws = wl.uneven_batch(seed=4, count=a.uneven_count)
    print(f"[uneven] {len(ws)} problems generated", file=sys.stderr, flush=True)
    npred = sum(w.m1 * w.m2 for w in ws)
    out = {"metric": "grid predictions/s, uneven batch of %d problems (one graph replay)" % len(ws),
           "unit": "grid predictions/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "config": {"workload": "uneven batch: grids from {128,256,384,512,1024}^2, n log-uniform in "
                                  "[500, 20000], L in {2,3,4}, nu in {0.5,1.5,2.5}, range U[0.05,0.3], nugget 0.01",
                      "problems": len(ws), "grid_points": npred, "n_max": max(w.sites.shape[0] for w in ws)}}
    res = {}
    # algorithmic bytes of one pass (one field per problem): the two FP64 triangles of every
    # solve (n^2 / 2 doubles each) and the prediction's three transform passes in the survey's
    # FP32-spectra model
    tri_bytes, conv_bytes = 0, 0
    for dtype in (("f32",) if a.no_fp64 else ("f32", "f64")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plans = []
        for i, w in enumerate(ws):
            plans.append(krig.plan_for(w, dtype))
            if dtype == "f32":
                sb = stage_bytes(plans[-1], 1, "s8d")
                tri_bytes += 8 * w.sites.shape[0] ** 2
                conv_bytes += sb["ROWS_FWD"] + sb["COLS_CONV"] + sb["ROWS_INV"]
            if i % 8 == 7:
                torch.cuda.synchronize()
                print(f"[uneven] {dtype}: {i + 1} plans, {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if not a.no_autotune:
            for i, p in enumerate(plans):
                p.autotune(1, with_adjoint=False)
                if i % 8 == 7:
                    print(f"[uneven] {dtype}: {i + 1} tuned, {time.perf_counter() - t1:.1f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ys = [torch.as_tensor(w.y, dtype=torch.float64, device=dev) for w in ws]
        outs = [p.empty(1, w.m1, w.m2) for p, w in zip(plans, ws)]
        # an explicit stream: a batch given the default (NULL) stream records and replays on a
        # stream of its own, which the timing events would not wait for
        st = torch.cuda.Stream(device=dev)
        st.wait_stream(torch.cuda.current_stream(dev))
        ctx = torch.cuda.stream(st)
        ctx.__enter__()
        bt = krig.Batch(plans, ys, outs, lanes=4)
        for _ in range(a.warmup):
            bt.launch()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record()
        for _ in range(a.steps):
            bt.launch()
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / a.steps
        # the same problems one plan after another, no graph
        torch.cuda.synchronize()
        s.record()
        for _ in range(a.steps):
            for p, y, o in zip(plans, ys, outs):
                p.predict(y, out=o)
        e.record()
        torch.cuda.synchronize()
        ms_eager = s.elapsed_time(e) / a.steps
        y_branches = [o.double().cpu().numpy() for o in outs]
        bt.close()
        # the persistent form: one work-queue launch per pass and kernel form
        bq = krig.Batch(plans, ys, outs, lanes=0)
        for _ in range(a.warmup):
            bq.launch()
        torch.cuda.synchronize()
        s.record()
        for _ in range(a.steps):
            bq.launch()
        e.record()
        torch.cuda.synchronize()
        ms_queue = s.elapsed_time(e) / a.steps
        same = all(np.array_equal(o.double().cpu().numpy(), yb) for o, yb in zip(outs, y_branches))
        bq.close()
        ctx.__exit__(None, None, None)
        torch.cuda.synchronize()
        res[dtype] = dict(ms=ms_queue, ms_branches=ms, ms_eager=ms_eager, setup_s=t1 - t0, tune_s=t2 - t1,
                          y=y_branches, persistent_bitwise_equal=same)
        del bt, plans, outs
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    r32 = res["f32"]
    r64 = res.get("f64", r32)
    errs = [float(np.max(np.abs(a_ - b_)) / np.max(np.abs(b_))) for a_, b_ in zip(r32["y"], r64["y"])]
    err = max(errs)
    worst = sorted(range(len(ws)), key=lambda i: -errs[i])[:5]
    out["worst_problems"] = [{"problem": ws[i].name, "rel_err": errs[i]} for i in worst]
    out["problems_over_1e-5"] = sum(e > 1e-5 for e in errs)
    # the faster of the two recorded forms is the figure; both are reported
    best = lambda r: min(r["ms"], r["ms_branches"])
    out.update({"value": npred / (best(r32) * 1e-3), "ms_per_step": best(r32), "steps": a.steps,
                "warmup": a.warmup, "dtype": "f64", "io_dtype": "f32", "scaling": "weak", "vs_baseline": None,
                "fp64_value": npred / (best(r64) * 1e-3), "fp64_ms_per_step": best(r64),
                "launch": ("persistent: one launch per pass and kernel form" if r32["ms"] <= r32["ms_branches"] else
                           "branches: every problem's own launches over 4 parallel branches") + ", one HIP graph",
                "persistent_ms_per_step": {"f32": r32["ms"], "f64": r64["ms"]},
                "branches_ms_per_step": {"f32": r32["ms_branches"], "f64": r64["ms_branches"]},
                "persistent_bitwise_equal_to_branches": {"f32": r32["persistent_bitwise_equal"],
                                                         "f64": r64["persistent_bitwise_equal"]},
                "eager_ms_per_step": {"f32": r32["ms_eager"], "f64": r64["ms_eager"]},
                "fp32_vs_fp64_rel_err": err,
                # whole pass against HBM: the triangles dominate (every problem's factor is read
                # once per solve, and the working set is far beyond the 256 MB last-level cache)
                "roofline": {"bound": "hbm", "kernel": "whole pass (every problem's FP64 triangular products "
                                                       "and transforms)",
                             "achieved": (tri_bytes + conv_bytes) / (best(r32) * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": (tri_bytes + conv_bytes) / (best(r32) * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "traffic": None, "bytes_per_pass": tri_bytes + conv_bytes, "triangle_bytes": tri_bytes,
                             "bytes_model": "two FP64 triangles of n^2/2 per solve; transforms in the FP32-spectra "
                                            "model"},
                "setup_s": {"f32": r32["setup_s"], "f64": r64["setup_s"]},
                "autotune_s": {"f32": r32["tune_s"], "f64": r64["tune_s"]}})
    print(json.dumps(out), flush=True)
    return 0


def interp_mode(a, torch, krig, wl, dev):
    """Off-grid predictions (krig_interp): the paper-sized mesh prediction (350x350, B fields,
    FP32 plan) interpolated to seeded uniform points with q x q local Lagrange stencils.
    Prints one JSON line."""
    w = wl.grad_batch(B=a.B)
    B, npts, q = a.B, a.interp_points, a.interp_q
    p = krig.plan_for(w, "f32")
    yhat = p.predict(torch.as_tensor(w.y, dtype=torch.float64, device=dev))
    rng = np.random.default_rng(99)
    pts_h = np.stack([w.x0 + rng.uniform(0, w.m1 - 1, npts) * w.dx, w.y0 + rng.uniform(0, w.m2 - 1, npts) * w.dy], 1)
    pts = torch.as_tensor(pts_h, dtype=torch.float64, device=dev)
    out = torch.empty(B, npts, dtype=torch.float32, device=dev)
    for _ in range(a.warmup):
        p.interp(yhat, pts, q, out=out)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(a.steps):
        p.interp(yhat, pts, q, out=out)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / a.steps
    # algorithmic bytes: the points once, every output once, the mesh prediction once
    nbytes = npts * 16 + B * npts * 4 + B * w.m1 * w.m2 * 4
    achieved = nbytes / (ms * 1e-3) / 1e9
    res = {"metric": "off-grid predictions/s (mesh prediction -> irregular points, local Lagrange q=%d)" % q,
           "value": B * npts / (ms * 1e-3), "unit": "off-grid predictions/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "io_dtype": "f32", "data": "synthetic",
           "config": {"workload": "off-grid interpolation: 350x350 mesh prediction of the paper-sized field, "
                                  "%d fields, %d seeded uniform points, %dx%d Lagrange stencils" % (B, npts, q, q),
                      "B": B, "points": npts, "q": q, "grid": [w.m1, w.m2]},
           "roofline": {"bound": "hbm", "kernel": "INTERP", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic("INTERP"),
                        "bytes_per_launch": nbytes, "avg_launch_ms": ms}}
    if not a.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle.interp import interp_points
        from oracle.rapid import Grid
        g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
        Yh = yhat.double().cpu().numpy()
        nf, npc = min(4, B), min(npts, 100_000)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            for b in range(nf):
                interp_points(g, Yh[b], pts_h[:npc], q)
            dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": nf * npc / dt, "unit": "off-grid predictions/s", "cores": 1, "kind": "oracle",
                               "host": host_cpu(),
                               "sample": f"{nf} fields x {npc} points, one thread, {dt:.1f} s"}
    print(json.dumps(res), flush=True)
    return 0


def caller_kvecs(w):
    """The --nonstat mode's input: a caller's nonstationary covariance vectors k_i[m] = C(g_m, s_i)
    at the neighbourhood nodes krig_set_kvec documents (anchor (floor((x - x0)/dx), floor((y -
    y0)/dy)), offsets (ox, oy) in {-L+1..L}^2, ox-major), for the caller's covariance model
    C(p, q) = sd(p) sd(q) exp(-|p - q| / range) with a smoothly varying sd.  A timing input only:
    set_kvec's cost does not depend on the values."""
    i0 = np.floor((w.sites[:, 0] - w.x0) / w.dx).astype(np.int64)
    j0 = np.floor((w.sites[:, 1] - w.y0) / w.dy).astype(np.int64)
    o = np.arange(-w.L + 1, w.L + 1)
    ox, oy = np.repeat(o, 2 * w.L), np.tile(o, 2 * w.L)
    gx = w.x0 + (i0[:, None] + ox[None, :]) * w.dx
    gy = w.y0 + (j0[:, None] + oy[None, :]) * w.dy
    sd = lambda x, y: 1.0 + 0.3 * np.sin(3.0 * x + 0.5) * np.cos(2.0 * y)
    sx, sy = w.sites[:, :1], w.sites[:, 1:]
    return sd(gx, gy) * sd(sx, sy) * w.sigma2 * np.exp(-np.hypot(gx - sx, gy - sy) / w.rho)


def nonstat_mode(a, torch, krig, wl, dev):
    """Nonstationary covariance vectors (krig_set_kvec) on the paper-sized field: weights
    from caller k_i (C(p, q) = sd(p) sd(q) k(p - q)), then the convolution of B fields'
    coefficients with them.  Prints one JSON line."""
    w = wl.grad_batch(B=a.B)
    kv = torch.as_tensor(caller_kvecs(w), dtype=torch.float64, device=dev)
    p = krig.plan_for(w, "f32")
    alpha = torch.as_tensor(np.random.default_rng(0).standard_normal((a.B, w.n)), dtype=torch.float64, device=dev)
    out = torch.empty(a.B, w.m1, w.m2, dtype=torch.float32, device=dev)

    def timed(fn):
        for _ in range(a.warmup):
            fn()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record()
        for _ in range(a.steps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / a.steps

    ms_kvec = timed(lambda: p.set_kvec(kv))
    ms_conv = timed(lambda: p.convolve(alpha, out=out))
    res = {"metric": "nonstationary k_i: weight updates (krig_set_kvec) and predictions with them",
           "value": a.B * w.m1 * w.m2 / (ms_conv * 1e-3), "unit": "grid predictions/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_conv, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "io_dtype": "f32", "data": "synthetic",
           "config": {"workload": "paper-sized field (n=1368, 350x350, L=3), caller k_i from "
                                  "sd(p) sd(q) exp(-|p - q| / range); B fields of coefficients", "B": a.B},
           "set_kvec_ms": ms_kvec, "weights_per_s": w.n / (ms_kvec * 1e-3)}
    print(json.dumps(res), flush=True)
    return 0


def csim_bytes(p, R, model="s8d"):
    """Algorithmic bytes per launch of the conditional-simulation stages (R realisations,
    (R + 1) / 2 complex pairs).  The sampler's column pass writes, per pair, the P1 torus rows
    the padded grid needs (Fs2 columns each) and reads sqrt(Lambda) once; its row pass reads them
    and writes two realisations; the residual kernel reads each realisation's field at the sites'
    neighbourhoods (at most the padded grid), the weights and data, and writes the residuals; the
    prediction passes are those of stage_bytes with B = R, the last adding the field.  Model "s8d":
    FP32 spectra and fields (the survey's model); "build": the plan's dtype for the sampler and the
    fields, the prediction passes' spectra as stage_bytes counts them."""
    P1, P2, n, M, m1, m2 = p.P1, p.P2, p.n, p.M, p.m1, p.m2
    Fs1, Fs2 = p.info("CE_F1"), p.info("CE_F2")
    npairs = (R + 1) // 2
    f32 = p.dtype_code == 1
    cz, t = (8, 4) if (model == "s8d" or f32) else (16, 8)
    sb = stage_bytes(p, R, model)
    return {
        "CSIM_CE": npairs * Fs2 * P1 * cz + (Fs2 // 2 + 1) * Fs1 * 8,
        "CSIM_ROWS": npairs * Fs2 * P1 * cz + R * P1 * P2 * t,
        "GATHER": R * (min(n * M, P1 * P2) * t + n * 8) + n * M * 8 + n * 8,
        "ROWS_FWD": sb["ROWS_FWD"],
        "COLS_CONV": sb["COLS_CONV"],
        "ROWS_INV": sb["ROWS_INV"] + R * m1 * m2 * t,
    }


def csim_mode(a, torch, krig, wl, dev):
    """Batched conditional simulation (krig_csim): R = 256 realisations on a 512 x 512 grid,
    n = 5000 uniform sites, Matern nu = 1.5, range 0.1, nugget 0.01, L = 4.  Each call draws
    R unconditional fields by circulant embedding, reads them at the sites through the
    neighbour weights and krigs the residuals.  Plan creation and one call per step are timed
    for the FP32 and FP64 plans.  Prints one JSON line."""
    w = wl.csim_batch(R=256)
    R, seed = w.extra["R"], w.extra["ce_seed"]
    y = torch.as_tensor(w.y[0], dtype=torch.float64, device=dev)
    per = {}
    for dtype in ("f32", "f64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = krig.plan_for(w, dtype)
        torch.cuda.synchronize()
        plan_ms = (time.perf_counter() - t0) * 1e3
        for _ in range(min(a.warmup, 5)):
            p.csim(R, seed, y)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record()
        for _ in range(a.steps):
            p.csim(R, seed, y)
        e.record()
        torch.cuda.synchronize()
        per[dtype] = {"plan_ms": plan_ms, "ms_per_call": s.elapsed_time(e) / a.steps}
        # per-stage kernel times (HIP events around each launch, same stream)
        p.timing(True)
        for _ in range(a.steps):
            p.csim(R, seed, y)
        st = p.timing_read()
        p.timing(False)
        avg = {k: v[0] / v[1] for k, v in st.items() if v[1] > 0}
        sb, sbb = csim_bytes(p, R, "s8d"), csim_bytes(p, R, "build")
        dom = max((k for k in sb if k in avg), key=lambda k: avg[k])
        per[dtype]["stage_avg_ms"] = {k: round(v, 4) for k, v in avg.items()}
        per[dtype]["stage_gbs"] = {k: round(sb[k] / (avg[k] * 1e-3) / 1e9, 1) for k in sb if k in avg}
        per[dtype]["stage_gbs_build"] = {k: round(sbb[k] / (avg[k] * 1e-3) / 1e9, 1) for k in sbb if k in avg}
        achieved = sb[dom] / (avg[dom] * 1e-3) / 1e9
        per[dtype]["roofline"] = {
            "bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic("CSIM_" + dom if not dom.startswith("CSIM") else dom),
            "bytes_per_launch": sb[dom], "bytes_model": "s8d: FP32 spectra and fields", "avg_launch_ms": avg[dom],
            "build_bytes_per_launch": sbb[dom], "build_frac": sbb[dom] / (avg[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS}
        p.close()
    ms = per["f32"]["ms_per_call"]
    res = {"metric": "conditional simulation: realisation grid values/s (R fields per call)",
           "value": R * w.m1 * w.m2 / (ms * 1e-3), "unit": "grid values/s", "n_gpus": 1, "steps": a.steps,
           "warmup": min(a.warmup, 5), "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "io_dtype": "f32", "data": "synthetic",
           "config": {"workload": "csim: R=256 realisations, 512x512 grid on [0,1]^2, n=5000 uniform sites, "
                                  "Matern nu=1.5 range 0.1 nugget 0.01, L=4 (M=64)", "R": R},
           "roofline": per["f32"]["roofline"],
           "per_dtype": per}
    print(json.dumps(res), flush=True)
    return 0


def mixture_mode(a, torch, krig, wl, dev):
    """Nonstationary mixture (krig_mixture) on the paper-sized field: two stationary
    components (the field's own Matern nu = 2.5, range 0.3 and a nu = 1.5, range 0.15 one)
    with weights cos^2 / sin^2 of x, B fields of coefficients.  Prints one JSON line."""
    import dataclasses
    w = wl.grad_batch(B=a.B)
    w2 = dataclasses.replace(w, sigma2=0.5, rho=0.15, nu=1.5)
    plans = [krig.plan_for(w, "f32"), krig.plan_for(w2, "f32")]
    lam = [lambda p: np.cos(1.5 * p[..., 0]) ** 2 + 0.1, lambda p: np.sin(1.5 * p[..., 0]) ** 2 + 0.1]
    X, Y = np.meshgrid(w.x0 + np.arange(w.m1) * w.dx, w.y0 + np.arange(w.m2) * w.dy, indexing="ij")
    nodes = np.stack([X, Y], -1)
    lam_sites = torch.as_tensor(np.stack([f(w.sites) for f in lam]), dtype=torch.float64, device=dev)
    lam_grid = torch.as_tensor(np.stack([f(nodes) for f in lam]), dtype=torch.float64, device=dev)
    alpha = torch.as_tensor(np.random.default_rng(0).standard_normal((a.B, w.n)), dtype=torch.float64, device=dev)
    out = torch.empty(a.B, w.m1, w.m2, dtype=torch.float32, device=dev)
    for _ in range(a.warmup):
        krig.mixture(plans, alpha, lam_sites, lam_grid, out=out)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(a.steps):
        krig.mixture(plans, alpha, lam_sites, lam_grid, out=out)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / a.steps
    res = {"metric": "grid predictions/s, nonstationary mixture of 2 stationary components",
           "value": a.B * w.m1 * w.m2 / (ms * 1e-3), "unit": "grid predictions/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "io_dtype": "f32", "data": "synthetic",
           "config": {"workload": "paper-sized field (n=1368, 350x350, L=3), components Matern(nu 2.5, range 0.3) and "
                                  "Matern(nu 1.5, range 0.15), weights cos^2 / sin^2 of x; B fields", "B": a.B,
                      "components": 2}}
    print(json.dumps(res), flush=True)
    return 0


def universal_mode(a, torch, krig, wl, dev):
    """Universal kriging (krig_predict_universal) on the paper-sized field: covariates
    (1, x, y, xy), B fields of data with a trend.  Prints one JSON line."""
    w = wl.grad_batch(B=a.B)
    p = krig.plan_for(w, "f32")
    design = lambda x, y: np.stack([np.ones_like(x), x, y, x * y])
    X, Y = np.meshgrid(w.x0 + np.arange(w.m1) * w.dx, w.y0 + np.arange(w.m2) * w.dy, indexing="ij")
    Xs = torch.as_tensor(design(w.sites[:, 0], w.sites[:, 1]), dtype=torch.float64, device=dev)
    Xg = torch.as_tensor(design(X, Y), dtype=torch.float64, device=dev)
    z = torch.as_tensor(w.y + np.array([1.0, 0.5, -0.5, 0.2]) @ design(w.sites[:, 0], w.sites[:, 1]),
                        dtype=torch.float64, device=dev)
    out = torch.empty(a.B, w.m1, w.m2, dtype=torch.float32, device=dev)

    def timed(fn):
        for _ in range(a.warmup):
            fn()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record()
        for _ in range(a.steps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / a.steps

    ms = timed(lambda: p.predict_universal(z, Xs, Xg, out=out))
    ms_plain = timed(lambda: p.predict(z, out=out))
    res = {"metric": "grid predictions/s, universal kriging (GLS trend in 4 covariates)",
           "value": a.B * w.m1 * w.m2 / (ms * 1e-3), "unit": "grid predictions/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "io_dtype": "f32", "data": "synthetic",
           "config": {"workload": "paper-sized field (n=1368, 350x350, L=3), covariates (1, x, y, xy), B fields",
                      "B": a.B, "covariates": 4},
           "plain_predict_ms": ms_plain}
    print(json.dumps(res), flush=True)
    return 0


def exact_mode(a, torch, krig, wl, dev):
    """The rapid predictor against exact kriging (the dense O(N n) sum, krig_predict_exact)
    on the paper-sized field with B fields, both on the GPU from the same coefficients:
    times, speedup and the approximation error.  Prints one JSON line."""
    w = wl.grad_batch(B=a.B)
    p = krig.plan_for(w, "f32")
    y = torch.as_tensor(w.y, dtype=torch.float64, device=dev)
    alpha = p.solve(y)
    out = torch.empty(a.B, w.m1, w.m2, dtype=torch.float32, device=dev)

    def timed(fn, steps):
        for _ in range(min(a.warmup, 3)):
            fn()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record()
        for _ in range(steps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / steps

    rapid_ms = timed(lambda: p.convolve(alpha, out=out), a.steps)
    rapid_full_ms = timed(lambda: p.predict(y, out=out), a.steps)
    exact_ms = timed(lambda: p.exact(alpha, out=out), max(3, a.steps // 4))
    solve_ms = timed(lambda: p.solve(y), a.steps)
    rapid = p.convolve(alpha).double()
    exact = p.exact(alpha).double()
    torch.cuda.synchronize()
    diff = (rapid - exact).abs()
    scale = exact.abs().amax(dim=(1, 2))
    npred = a.B * w.m1 * w.m2
    res = {"metric": "grid predictions/s, rapid predictor vs exact kriging on the same GPU",
           "value": npred / (rapid_ms * 1e-3), "unit": "grid predictions/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": rapid_ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "io_dtype": "f32", "data": "synthetic",
           "config": {"workload": "paper-sized field (n=1368 sites, 350x350, L=3, Matern nu=2.5 range 0.3), "
                                  "B fields; rapid: scatter + FFT convolution, exact: sum over all sites",
                      "B": a.B, "n": w.n, "grid": [w.m1, w.m2]},
           "exact_ms": exact_ms, "exact_value": npred / (exact_ms * 1e-3),
           "exact_pair_evals_per_s": w.m1 * w.m2 * w.n / (exact_ms * 1e-3),
           "speedup_rapid_over_exact": exact_ms / rapid_ms,
           "with_solve": {"solve_ms": solve_ms, "rapid_ms": rapid_full_ms, "exact_ms": solve_ms + exact_ms,
                          "speedup": (solve_ms + exact_ms) / rapid_full_ms},
           "approximation_error": {"max_abs_rel_to_max": float((diff.amax(dim=(1, 2)) / scale).max()),
                                   "mean_abs": float(diff.mean()), "max_abs": float(diff.max())}}
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = exact_cpu_baseline(w)
    print(json.dumps(res), flush=True)
    return 0


def exact_cpu_baseline(w):
    """The oracle's rapid (FFT form) and exact predictions of one field on one host core."""
    from threadpoolctl import threadpool_limits

    from oracle.exact import ExactKriging
    from oracle.matern import Matern
    from oracle.rapid import Grid, RapidPredictor, lag_quadrant, rapid_fft
    g = Grid(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L)
    k = Matern(w.sigma2, w.rho, w.nu, w.tau2)
    with threadpool_limits(limits=1):
        rp = RapidPredictor(g, k, w.sites)
        ek = ExactKriging(w.sites, k)
        lag = lag_quadrant(g, k)
        c = ek.coef(w.y[0])
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            rapid_fft(g, lag, rp.cstar(c))
        t_rapid = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        ek.predict_at(g.nodes(), c)
        t_exact = time.perf_counter() - t0
    return {"value": w.m1 * w.m2 / t_rapid, "unit": "grid predictions/s", "cores": 1, "kind": "oracle",
            "sample": f"one field: the oracle's rapid prediction (FFT form, {reps} runs) and its exact prediction "
                      f"(dense sum over the {w.n} sites, {t_exact:.1f} s)",
            "exact_value": w.m1 * w.m2 / t_exact, "speedup_rapid_over_exact": t_exact / t_rapid,
            "host": host_cpu()}


# phi(r) = 0.7 for the smoothness levels of the factorial study (r K_1(r) for nu = 1): the
# study fixes the distance at which the correlation falls to 0.7, so range = that distance / R07[nu]
R07 = {0.5: 0.3566749439387324, 1.0: 0.7766915961392014, 1.5: 1.0973492107034915}


def table_a2_model(coef, nu, L, m, tau2):
    """Fitted log10 mean absolute error of Appendix A, Table A2 for one factor combination."""
    t = coef["(Intercept)"]
    if nu != 0.5:
        sn = "smoothness1" if nu == 1.0 else "smoothness1.5"
        t += coef[sn] + (coef[f"{sn}:NN{L}"] if L != 2 else 0.0)
    if L != 2:
        t += coef[f"NN{L}"]
    if m != 100:
        t += coef[f"nGrid{m}"]
    if tau2 != 0.01:
        t += coef[f"nugget{tau2}"]
    return t


def accuracy_mode(a, torch, krig, wl, dev):
    """The paper's factorial accuracy study (Section 3, Appendix A) at the levels the GPU path
    supports, as a batch of problems on the GPU: for every combination of n, range, smoothness,
    nugget, L and grid, seeded uniform site sets and data, the rapid prediction against exact
    kriging (krig_exact_at) at five nodes from the centre to the corner.  The log10 mean
    absolute error per case is compared with the fitted model of Table A2.  One JSON line."""
    coef = {}
    with open(os.path.join(ROOT, "tests", "golden", "tableA2_coef.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k_, v_ = line.split()
                coef[k_] = float(v_)
    levels = {"n": (200, 500, 1500), "d07": (0.2, 0.4, 0.8), "nu": (0.5, 1.0, 1.5), "tau2": (0.01, 0.1, 0.5),
              "L": (2, 4, 8), "m": (100, 350, 500)}
    rng = np.random.default_rng(27)
    cases = []
    t0 = time.perf_counter()
    for m in levels["m"]:
        h = 1.0 / (m - 1)
        ab = [(m // 2, m // 2), (m // 4, m // 4), (0, 0), (m // 2, 0), (m - 1, m // 2)]
        idx = torch.as_tensor([i * m + j for i, j in ab], device=dev)
        pts = torch.as_tensor([[i * h, j * h] for i, j in ab], dtype=torch.float64, device=dev)
        for L in levels["L"]:
            for nu in levels["nu"]:
                for tau2 in levels["tau2"]:
                    for d07 in levels["d07"]:
                        for n in levels["n"]:
                            rho = d07 / R07[nu]
                            errs, failed = [], []
                            for _ in range(a.accuracy_reps):
                                sites = wl.sites_uniform(rng, n)
                                y = wl.add_nugget(rng, wl.rff_draw(rng, sites, 1.0, rho, nu), tau2)
                                try:
                                    p = krig.Plan(m, m, 0.0, 0.0, h, h, L, 1.0, rho, nu, tau2, sites, "f64")
                                except krig.KrigError as e:  # e.g. a non-positive pivot in K_N
                                    failed.append(e.status)
                                    continue
                                al = p.solve(torch.as_tensor(y, dtype=torch.float64, device=dev))
                                rapid = p.convolve(al).reshape(-1)[idx]
                                exact = p.exact_at(al, pts)[0]
                                errs.append((rapid - exact).abs().cpu().numpy())
                                p.close()
                            if not errs:
                                cases.append({"n": n, "d07": d07, "nu": nu, "tau2": tau2, "L": L, "m": m,
                                              "failed": failed})
                                continue
                            got = float(np.log10(np.mean(errs)))
                            cases.append({"n": n, "d07": d07, "nu": nu, "tau2": tau2, "L": L, "m": m,
                                          "log10_mean_abs_err": round(got, 3),
                                          "table_a2": round(table_a2_model(coef, nu, L, m, tau2), 3)})
    secs = time.perf_counter() - t0
    failed = [c for c in cases if "failed" in c]
    cases_ok = [c for c in cases if "failed" not in c]
    dev_ = np.array([c["log10_mean_abs_err"] - c["table_a2"] for c in cases_ok])
    got_all = np.array([c["log10_mean_abs_err"] for c in cases_ok])

    def effect(key, lev, base):
        sel = lambda v: np.array([c[key] == v for c in cases_ok])
        return round(float(got_all[sel(lev)].mean() - got_all[sel(base)].mean()), 3)

    effects = {"nu1": [effect("nu", 1.0, 0.5), coef["smoothness1"]], "nu1.5": [effect("nu", 1.5, 0.5), coef["smoothness1.5"]],
               "L4": [effect("L", 4, 2), coef["NN4"]], "L8": [effect("L", 8, 2), coef["NN8"]],
               "grid350": [effect("m", 350, 100), coef["nGrid350"]], "grid500": [effect("m", 500, 100), coef["nGrid500"]],
               "nugget0.1": [effect("tau2", 0.1, 0.01), coef["nugget0.1"]],
               "nugget0.5": [effect("tau2", 0.5, 0.01), coef["nugget0.5"]],
               "n500": [effect("n", 500, 200), None], "n1500": [effect("n", 1500, 200), None],
               "d07_0.4": [effect("d07", 0.4, 0.2), None], "d07_0.8": [effect("d07", 0.8, 0.2), None]}
    res = {"metric": "factorial accuracy study: |log10 mean abs error (rapid vs exact) - Table A2 model|, mean over cases",
           "value": float(np.abs(dev_).mean()), "unit": "decades", "n_gpus": 1, "higher_is_better": False,
           "data": "synthetic", "dtype": "f64",
           "config": {"workload": "factorial: n {200,500,1500} x correlation-0.7 distance {0.2,0.4,0.8} x nu {0.5,1,1.5} "
                                  "x nugget {0.01,0.1,0.5} x L {2,4,8} x grid {100,350,500}^2 on [0,1]^2, sigma2 = 1; "
                                  f"{a.accuracy_reps} seeded site sets per case; errors at five nodes from centre to corner",
                      "cases": len(cases), "site_sets_per_case": a.accuracy_reps},
           "seconds": secs, "problems_per_s": len(cases) * a.accuracy_reps / secs,
           "deviation_from_table_a2": {"mean": float(dev_.mean()), "rms": float(np.sqrt((dev_ ** 2).mean())),
                                       "max_abs": float(np.abs(dev_).max()),
                                       "within_one_decade": float((np.abs(dev_) < 1.0).mean())},
           "main_effects_vs_table_a2": effects, "failed_cases": len(failed),
           "cases": cases}
    print(json.dumps(res), flush=True)
    return 0


def convergence_mode(a, torch, krig, wl, dev):
    """Section 3.2 / Table 2 on the GPU: the error Lambda of the interpolated covariance
    (krig_kernel_at) against the exact one (krig_exact_at with a unit coefficient), as a
    supremum over [0,1]^2 (a 121 x 121 lattice plus an 81 x 81 patch around the site), for
    the Figure 5 set-up (range 0.25, L = 2, one site centred in the central grid box) on
    grids of 20^2 .. 140^2; the fitted slopes against the inverse fill distance are
    compared with the paper's.  Prints one JSON line."""
    gold = {}
    with open(os.path.join(ROOT, "tests", "golden", "table2_slopes.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k_, v_ = line.split()
                gold[float(k_)] = float(v_)
    one = torch.ones(1, 1, dtype=torch.float64, device=dev)
    ms = (20, 30, 40, 60, 80, 100, 140)
    out = {}
    t0 = time.perf_counter()
    for nu in (0.5, 1.0, 1.5, 2.5):
        lams, inv = [], []
        for m in ms:
            h = 1.0 / (m - 1)
            c = (m - 1) // 2
            s_ = np.array([[(c + 0.5) * h, (c + 0.5) * h]])
            p = krig.Plan(m, m, 0.0, 0.0, h, h, 2, 1.0, 0.25, nu, 0.0, s_, "f64")
            g1 = np.linspace(0, 1, 121)
            X, Y = np.meshgrid(g1, g1, indexing="ij")
            g2 = np.linspace(-3 * h, 3 * h, 81)
            U, V = np.meshgrid(g2, g2, indexing="ij")
            pts = torch.as_tensor(np.concatenate([np.stack([X.ravel(), Y.ravel()], 1),
                                                  s_ + np.stack([U.ravel(), V.ravel()], 1)]), device=dev)
            lams.append((p.kernel_at(0, pts) - p.exact_at(one, pts)[0]).abs().max().item())
            inv.append(1.0 / (0.5 * np.hypot(h, h)))
            p.close()
        slope = float(-np.polyfit(np.log10(inv), np.log10(lams), 1)[0])
        out[str(nu)] = {"lambda": lams, "slope": round(slope, 3), "table2": gold[nu]}
    res = {"metric": "Table 2 convergence: fitted order of the kernel approximation error vs 1/fill distance",
           "value": float(np.mean([abs(v["slope"] - v["table2"]) for v in out.values()])),
           "unit": "mean |slope - Table 2|", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
           "dtype": "f64", "config": {"workload": "Figure 5 set-up: [0,1]^2, Matern range 0.25, L = 2, one site "
                                                  "centred in the central box, grids " + ",".join(f"{m}^2" for m in ms),
                                      "nu": [0.5, 1.0, 1.5, 2.5]},
           "grids": list(ms), "by_nu": out, "seconds": time.perf_counter() - t0}
    print(json.dumps(res), flush=True)
    return 0


def device_copy_gbs(torch, dev, mib=1024, reps=10):
    """Bandwidth of a plain device-to-device copy of `mib` MiB: (read + write bytes) / time."""
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        dst.copy_(src)
    e.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * reps / (s.elapsed_time(e) * 1e-3) / 1e9
    del src, dst
    return round(gbs, 1)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed steps first; about 40 ms of sustained work settles the GPU clocks")
    ap.add_argument("--B", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-fields", type=int, default=16)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep plan_create's launch shapes")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of the step recorded as a HIP graph instead of the call loop")
    ap.add_argument("--uneven", action="store_true", help="time the 64-problem uneven batch instead")
    ap.add_argument("--uneven-count", type=int, default=64)
    ap.add_argument("--interp", action="store_true", help="time off-grid predictions (krig_interp) instead")
    ap.add_argument("--nonstat", action="store_true", help="time weights from caller k_i (krig_set_kvec) instead")
    ap.add_argument("--mixture", action="store_true", help="time a two-component nonstationary mixture instead")
    ap.add_argument("--csim", action="store_true", help="time batched conditional simulation (R = 256) instead")
    ap.add_argument("--universal", action="store_true", help="time universal kriging with a GLS trend instead")
    ap.add_argument("--exact", action="store_true", help="time the rapid predictor against exact kriging instead")
    ap.add_argument("--accuracy", action="store_true",
                    help="run the factorial accuracy study (rapid vs exact kriging, against Table A2) instead")
    ap.add_argument("--accuracy-reps", type=int, default=2, help="site sets per factorial case")
    ap.add_argument("--convergence", action="store_true",
                    help="measure the Table 2 convergence slopes of the kernel approximation instead")
    ap.add_argument("--interp-points", type=int, default=1_000_000)
    ap.add_argument("--interp-q", type=int, default=4)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}); the batch axis would shard with no "
              "communication, see the design notes.", file=sys.stderr)
        return 2

    import torch

    import paper_2605_29284_amd as krig
    import workloads as wl

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    if a.calibrate_copy_mib:
        n = a.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):  # a plain elementwise kernel: reads and writes 4n bytes each
            torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": 4 * n, "copies": 3}), flush=True)
        return 0
    if a.uneven:
        return uneven(a, torch, krig, wl, dev)
    if a.interp:
        return interp_mode(a, torch, krig, wl, dev)
    if a.nonstat:
        return nonstat_mode(a, torch, krig, wl, dev)
    if a.mixture:
        return mixture_mode(a, torch, krig, wl, dev)
    if a.csim:
        return csim_mode(a, torch, krig, wl, dev)
    if a.universal:
        return universal_mode(a, torch, krig, wl, dev)
    if a.exact:
        return exact_mode(a, torch, krig, wl, dev)
    if a.accuracy:
        return accuracy_mode(a, torch, krig, wl, dev)
    if a.convergence:
        return convergence_mode(a, torch, krig, wl, dev)
    w = wl.grad_batch(B=a.B)
    B = a.B

    def setup(dtype):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = krig.plan_for(w, dtype)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tuned = None if a.no_autotune else p.autotune(B, with_adjoint=True)
        torch.cuda.synchronize()
        return p, (t1 - t0) * 1e3, (time.perf_counter() - t1) * 1e3, tuned

    y = torch.as_tensor(w.y, dtype=torch.float64, device=dev)

    def buffers(p):
        td = p.tdtype
        return dict(alpha=torch.empty(B, w.n, dtype=torch.float64, device=dev), saved=p.new_saved(B),
                    yhat=torch.empty(B, w.m1, w.m2, dtype=td, device=dev),
                    dy=torch.empty(B, w.n, dtype=torch.float64, device=dev),
                    dlag=torch.empty(w.m1 + w.L, w.m2 + w.L, dtype=td, device=dev))

    def run(p, bf, g, steps, hot=False):
        for _ in range(steps):
            if hot:  # alpha given: scatter + convolution and its adjoint only
                p.convolve(bf["alpha"], saved=bf["saved"], out=bf["yhat"])
                p.adjoint(g, alpha=bf["alpha"], saved=bf["saved"], want_dy=False, dlag_out=bf["dlag"])
            else:
                p.predict(y, alpha_out=bf["alpha"], saved=bf["saved"], out=bf["yhat"])
                p.adjoint(g, alpha=bf["alpha"], saved=bf["saved"], dy_out=bf["dy"], dlag_out=bf["dlag"])

    def timed(p, bf, g, steps, hot=False, graph=None):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record()
        if graph is None:
            run(p, bf, g, steps, hot)
        else:
            for _ in range(steps):
                graph.replay()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / steps

    def record(p, bf, g, hot=False):
        # one step's launches recorded as a HIP graph (every kernel runs on each replay;
        # the buffers are the same ones the eager loop uses)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            run(p, bf, g, 1, hot)
        torch.cuda.synchronize()
        return graph

    mask = torch.as_tensor(w.extra["mask"], device=dev)
    res = {}
    for dtype in (("f32",) if a.no_fp64 else ("f32", "f64")):
        p, setup_ms, tune_ms, tuned = setup(dtype)
        bf = buffers(p)
        p.predict(y, alpha_out=bf["alpha"], saved=bf["saved"], out=bf["yhat"])
        g = (2.0 * mask.to(p.tdtype) * bf["yhat"]).contiguous()  # upstream gradient, fixed over the steps
        run(p, bf, g, a.warmup)
        eager_ms = timed(p, bf, g, a.steps)
        eager_hot_ms = timed(p, bf, g, a.steps, hot=True)
        gr, gh = record(p, bf, g), record(p, bf, g, hot=True)
        for _ in range(a.warmup):
            gr.replay()
        graph_ms = timed(p, bf, g, a.steps, graph=gr)
        graph_hot_ms = timed(p, bf, g, a.steps, hot=True, graph=gh)
        del gr, gh
        ms, hot_ms = (graph_ms, graph_hot_ms) if a.graph else (eager_ms, eager_hot_ms)
        # per-stage kernel times (HIP events around each launch, same stream)
        p.timing(True)
        run(p, bf, g, a.steps)
        stages = p.timing_read()
        p.timing(False)
        run(p, bf, g, 1)
        torch.cuda.synchronize()
        res[dtype] = dict(plan=p, ms=ms, graph_ms=graph_ms, hot_ms=hot_ms, setup_ms=setup_ms, tune_ms=tune_ms, tuned=tuned, stages=stages,
                          yhat=bf["yhat"].double().cpu().numpy(), dy=bf["dy"].cpu().numpy(),
                          dlag=bf["dlag"].double().cpu().numpy())

    r32 = res["f32"]
    p32 = r32["plan"]
    copy_gbs = device_copy_gbs(torch, dev)
    npred = B * w.m1 * w.m2
    value = npred / (r32["ms"] * 1e-3)
    # dominant single-kernel stage and its roofline: the survey's FP32-spectra byte model, with
    # the bytes this build's kernels move (FP64 spectra) beside it
    sb = stage_bytes(p32, B, "s8d")
    sbb = stage_bytes(p32, B, "build")
    avg = {k: (v[0] / v[1]) for k, v in r32["stages"].items() if v[1] > 0}
    dom = max((k for k in sb if k in avg), key=lambda k: avg[k])
    achieved = sb[dom] / (avg[dom] * 1e-3) / 1e9
    graded = [k for k in sb if k in avg]  # scatter, transform and gather passes
    graded_s = sum(avg[k] * r32["stages"][k][1] / a.steps for k in graded) * 1e-3
    out = {
        "metric": "grid predictions/s fwd+adjoint, FP32 vs FP64 at rel err <=1e-5; % HBM peak",
        "value": value,
        "unit": "grid predictions/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r32["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # both plans compute in FP64; the FP32 plan's lag, g, y_hat and d lag are FP32, and its
        # adjoint stores the upstream gradient's row spectra and the lag-gradient partials in FP32
        "dtype": "f64",
        "io_dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "grad-batch: paper-sized field, n=1368 sites on [0,2]x[0,1], Matern nu=2.5 "
                               "range 0.3 nugget 0.05, 350x350 grid, L=3 (M=36), B=16 fields, "
                               "forward (y->y_hat) + adjoint (g->dy, dlag)",
                   "B": B, "n": w.n, "grid": [w.m1, w.m2], "L": w.L, "fft": [p32.F1, p32.F2]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(dom),
                     "bytes_per_launch": sb[dom], "bytes_model": "s8d: FP32 spectra (the survey's model)",
                     "avg_launch_ms": avg[dom],
                     "build_bytes_per_launch": sbb[dom],
                     "build_frac": sbb[dom] / (avg[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "build_bytes_model": "the bytes this build's kernels move: FP64 spectra between the passes"},
        # every scatter, transform and gather pass of the step together (FP64 solves and the lag-gradient
        # tail excluded): s8d bytes over their summed kernel time
        "graded_passes": {"bytes_s8d": sum(sb[k] for k in graded), "ms": graded_s * 1e3,
                          "gbs": sum(sb[k] for k in graded) / graded_s / 1e9,
                          "frac": sum(sb[k] for k in graded) / graded_s / 1e9 / HBM_PEAK_GBS,
                          "build_frac": sum(sbb[k] for k in graded) / graded_s / 1e9 / HBM_PEAK_GBS,
                          "bytes_per_prediction_s8d": sum(sb[k] for k in graded) / npred},
        "launch": "HIP graph replay of one recorded step" if a.graph else "call loop",
        # the same step recorded once as a HIP graph and replayed (on this stack the graph
        # is not faster than the call loop's launches)
        "graph_ms_per_step": r32["graph_ms"],
        "hot_path_value": npred / (r32["hot_ms"] * 1e-3),
        "setup_ms": r32["setup_ms"],
        "autotune_ms": r32["tune_ms"],
        "launch_shapes": r32["tuned"],
        "stage_avg_ms": {k: round(v, 5) for k, v in avg.items()},
        "stage_calls_per_step": {k: v[1] / a.steps for k, v in r32["stages"].items() if v[1] > 0},
        # a plain device-to-device copy on the same GPU (reads + writes), beside the HBM peak
        "device_copy_gbs": copy_gbs,
        "stage_gbs": {k: round(sb[k] / (avg[k] * 1e-3) / 1e9, 1) for k in sb if k in avg},
        "stage_gbs_build": {k: round(sbb[k] / (avg[k] * 1e-3) / 1e9, 1) for k in sbb if k in avg},
    }
    if "f64" in res:
        r64 = res["f64"]
        rel = lambda x, y: float(np.max(np.abs(x - y)) / np.max(np.abs(y)))
        out["fp64_value"] = npred / (r64["ms"] * 1e-3)
        out["fp64_ms_per_step"] = r64["ms"]
        out["fp64_stage_avg_ms"] = {k: round(v[0] / v[1], 5) for k, v in r64["stages"].items() if v[1] > 0}
        out["fp32_vs_fp64_rel_err"] = {
            "yhat": max(rel(r32["yhat"][b], r64["yhat"][b]) for b in range(B)),
            "dy": rel(r32["dy"], r64["dy"]), "dlag": rel(r32["dlag"], r64["dlag"])}
    if not a.no_cpu_baseline:
        out["cpu_baseline"], ref = cpu_baseline(w, a.cpu_fields)
        # errors against the FP64 oracle on identical inputs (after all timings: the oracle's
        # weights are injected into the plans)
        out["max_rel_err_vs_oracle"] = {d: oracle_errors(torch, krig, w, res[d]["plan"], ref, dev) for d in res}
        out["max_rel_err_vs_oracle"]["inputs"] = (
            f"fields 0..{len(ref['yhat']) - 1}; the oracle's weights, data and FP32-rounded upstream gradient")
        out["max_rel_err_vs_oracle"]["bars"] = {"f32": {"yhat": 1e-5, "dy": 1e-6, "dlag": 1e-5},
                                                "f64": {"yhat": 1e-12}}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
