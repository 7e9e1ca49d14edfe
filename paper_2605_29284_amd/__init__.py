"""Python binding of libkrig, the GPU rapid Kriging predictor (Li, Fasshauer & Nychka).

Argument marshalling only: every step runs in the HIP kernels of libkrig.so,
called through its C ABI (include/krig.h).  PyTorch supplies device memory and
the current stream.  There is no CPU fallback: importing the binding without a
built library, or calling it without a GPU, raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkrig.so")

KRIG_F32 = 1
KRIG_F64 = 2

INFO = dict(N=1, M=2, P1=3, P2=4, F1=5, F2=6, H2=7, LDH=8, SAVED_PER_FIELD=9, KN_STATUS=10,
            PIVOT=11, DTYPE=12, CE_CLAMPED=13, DLAG_GROUP=14, CE_F1=15, CE_F2=16, NL_ROWS64=17,
            NL_COLS64=18, FFT_R1=19, FFT_R2=20, FFT_R3=21, FFT_VARIANTS_ROWS=22, FFT_VARIANTS_COLS=23,
            FFT_VARIANT_ROWS=24, FFT_VARIANT_COLS=25, SOLVE_NOALLOC_MAX_B=26, FILTER_SETUP=27, COLS_PAIR=28, SCATTER=29)
FILTER = dict(reflected=0, centered=1)
TUNE = dict(DLAG_GROUP=1, NL_ROWS64=2, NL_COLS64=3, FFT_ROWS=4, FFT_COLS=5, COLS_PAIR=6, SCATTER=7)

STATUS = {0: "KRIG_OK", -1: "KRIG_EINVAL", -2: "KRIG_EDOMAIN", -3: "KRIG_ENOTSPD", -4: "KRIG_ECE",
          -5: "KRIG_ENOMEM", -6: "KRIG_EHIP", -7: "KRIG_EUNSUPPORTED"}

EXPORTS = ["krig_plan_create", "krig_plan_destroy", "krig_plan_info", "krig_set_stream", "krig_weights",
           "krig_set_weights", "krig_set_kvec", "krig_lag", "krig_filter", "krig_solve", "krig_solve_noalloc", "krig_scatter", "krig_convolve", "krig_predict",
           "krig_predict_adjoint", "krig_csim", "krig_interp", "krig_predict_exact", "krig_exact_at", "krig_kernel_at", "krig_mixture", "krig_predict_universal", "krig_plan_tune", "krig_plan_autotune", "krig_predict_many", "krig_batch_create",
           "krig_batch_launch", "krig_batch_destroy", "krig_timing_enable", "krig_timing_read", "krig_strerror"]

STAGES = ["ROWS_FWD", "COLS_CONV", "ROWS_INV", "ADJ_ROWS_FWD", "ADJ_COLS", "ADJ_ROWS_INV", "GATHER", "SOLVE",
          "DLAG_TAIL", "CSIM_CE", "CSIM_ROWS"]


class KrigError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({_strerror(status)})")


class _Grid(ctypes.Structure):
    _fields_ = [("m1", ctypes.c_int32), ("m2", ctypes.c_int32), ("x0", ctypes.c_double),
                ("y0", ctypes.c_double), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("L", ctypes.c_int32)]


class _Matern(ctypes.Structure):
    _fields_ = [("sigma2", ctypes.c_double), ("range", ctypes.c_double), ("nu", ctypes.c_double),
                ("tau2", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libkrig.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2605_29284_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    sig = {
        "krig_plan_create": [ctypes.POINTER(vp), ctypes.POINTER(_Grid), ctypes.POINTER(_Matern), i32, dp, i32, vp],
        "krig_plan_destroy": [vp],
        "krig_plan_info": [vp, i32, ctypes.POINTER(i64)],
        "krig_set_stream": [vp, vp],
        "krig_weights": [vp, dp, dp],
        "krig_set_weights": [vp, dp, dp],
        "krig_set_kvec": [vp, dp],
        "krig_lag": [vp, dp],
        "krig_filter": [vp, i32, dp],
        "krig_solve": [vp, i32, dp, dp],
        "krig_solve_noalloc": [vp, i32, dp, dp],
        "krig_scatter": [vp, i32, dp, dp],
        "krig_convolve": [vp, i32, dp, dp, dp, dp],
        "krig_predict": [vp, i32, dp, dp, dp, dp, dp],
        "krig_predict_adjoint": [vp, i32, dp, dp, dp, dp, dp, dp],
        "krig_csim": [vp, i32, ctypes.c_uint64, dp, dp],
        "krig_interp": [vp, i32, dp, i32, dp, i32, dp],
        "krig_predict_exact": [vp, i32, dp, dp],
        "krig_exact_at": [vp, i32, dp, i32, dp, dp],
        "krig_kernel_at": [vp, i32, i32, dp, dp],
        "krig_mixture": [ctypes.POINTER(vp), i32, i32, dp, dp, dp, dp, vp],
        "krig_predict_universal": [vp, i32, dp, i32, dp, dp, dp, dp, dp],
        "krig_plan_tune": [vp, i32, i64],
        "krig_plan_autotune": [vp, i32, i32],
        "krig_predict_many": [ctypes.POINTER(vp), i32, ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.POINTER(vp), vp],
        "krig_batch_create": [ctypes.POINTER(vp), ctypes.POINTER(vp), i32, ctypes.POINTER(i32), ctypes.POINTER(vp),
                              ctypes.POINTER(vp), i32, vp],
        "krig_batch_launch": [vp, vp],
        "krig_batch_destroy": [vp],
        "krig_timing_enable": [vp, i32],
        "krig_timing_read": [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.krig_strerror.argtypes = [ctypes.c_int]
    lib.krig_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _strerror(status: int) -> str:
    try:
        return load_library().krig_strerror(status).decode()
    except Exception:  # library missing: message only
        return "?"


def _check(status: int, what: str):
    if status != 0:
        raise KrigError(status, what)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Plan:
    """One site set, Matern kernel, grid and dtype (see krig_plan_create)."""

    def __init__(self, m1: int, m2: int, x0: float, y0: float, dx: float, dy: float, L: int,
                 sigma2: float, rho: float, nu: float, tau2: float, sites, dtype: str = "f32",
                 device: str = "cuda:0"):
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("libkrig needs a GPU (no device visible)")
        self.lib = load_library()
        self.device = torch.device(device)
        self.dtype_code = {"f32": KRIG_F32, "f64": KRIG_F64}[dtype]
        self.tdtype = torch.float32 if dtype == "f32" else torch.float64
        self.m1, self.m2, self.L = int(m1), int(m2), int(L)
        s = np.ascontiguousarray(np.asarray(sites, dtype=np.float64))
        if s.ndim != 2 or s.shape[1] != 2:
            raise ValueError("sites must be n x 2")
        self.n = s.shape[0]
        g = _Grid(self.m1, self.m2, x0, y0, dx, dy, self.L)
        k = _Matern(sigma2, rho, nu, tau2)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = torch.cuda.current_stream(self.device).cuda_stream
            _check(self.lib.krig_plan_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(k), self.n,
                                             s.ctypes.data, self.dtype_code, st), "krig_plan_create")
        self.h = h
        self.M = self.info("M")
        self.P1, self.P2 = self.info("P1"), self.info("P2")
        self.F1, self.F2 = self.info("F1"), self.info("F2")
        self.saved_per_field = self.info("SAVED_PER_FIELD")

    # -- plumbing ---------------------------------------------------------------------
    def __del__(self):
        try:
            if getattr(self, "h", None) and self.h.value:
                self.lib.krig_plan_destroy(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass

    def close(self):
        self.__del__()

    def info(self, key: str) -> int:
        v = ctypes.c_int64()
        _check(self.lib.krig_plan_info(self.h, INFO[key], ctypes.byref(v)), "krig_plan_info")
        return int(v.value)

    def _stream(self):
        st = self.torch.cuda.current_stream(self.device).cuda_stream
        _check(self.lib.krig_set_stream(self.h, st), "krig_set_stream")

    def _t(self, x, dtype, shape, name):
        t = self.torch
        if not isinstance(x, t.Tensor) or x.device != self.device or x.dtype != dtype or not x.is_contiguous():
            raise TypeError(f"{name}: expected a contiguous {dtype} tensor on {self.device}")
        if tuple(x.shape) != tuple(shape):
            raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(x.shape)}")
        return x

    def _batch(self, x, last, name, dtype):
        if x.dim() == len(last):
            x = x.unsqueeze(0)
        return self._t(x, dtype, (x.shape[0],) + tuple(last), name)

    def empty(self, *shape, dtype=None):
        return self.torch.empty(*shape, dtype=dtype or self.tdtype, device=self.device)

    # -- entry points -----------------------------------------------------------------
    def weights(self) -> Tuple["torch.Tensor", "torch.Tensor"]:
        a = self.empty(self.n, 2, dtype=self.torch.int32)
        w = self.empty(self.n, self.M, dtype=self.torch.float64)
        self._stream()
        _check(self.lib.krig_weights(self.h, a.data_ptr(), w.data_ptr()), "krig_weights")
        return a, w

    def set_weights(self, anchor, W):
        self._t(anchor, self.torch.int32, (self.n, 2), "anchor")
        self._t(W, self.torch.float64, (self.n, self.M), "W")
        self._stream()
        _check(self.lib.krig_set_weights(self.h, anchor.data_ptr(), W.data_ptr()), "krig_set_weights")

    def set_kvec(self, kvec):
        """Weights from caller covariance vectors k_i [n][M] FP64 (krig_set_kvec):
        W_i = K_N^{-1} k_i with the plan's stationary K_N."""
        kvec = self._t(kvec, self.torch.float64, (self.n, self.M), "kvec")
        self._stream()
        _check(self.lib.krig_set_kvec(self.h, kvec.data_ptr()), "krig_set_kvec")

    def lag(self):
        out = self.empty(self.m1 + self.L, self.m2 + self.L)
        self._stream()
        _check(self.lib.krig_lag(self.h, out.data_ptr()), "krig_lag")
        return out

    def filter(self, setup: str = None):
        """The filter spectrum [H2][F1] FP64 (scaled by 1/(F1 F2)); setup "reflected" or "centered"
        rebuilds it first (krig_filter)."""
        out = self.empty(self.info("H2"), self.F1, dtype=self.torch.float64)
        s = self.info("FILTER_SETUP") if setup is None else FILTER[setup]
        self._stream()
        _check(self.lib.krig_filter(self.h, s, out.data_ptr()), "krig_filter")
        return out

    def solve(self, y, out=None):
        """krig_solve; out may be y itself (an in-place solve)."""
        y = self._batch(y, (self.n,), "y", self.torch.float64)
        if out is None:
            out = self.empty(y.shape[0], self.n, dtype=self.torch.float64)
        else:
            out = self._t(out, self.torch.float64, (y.shape[0], self.n), "out")
        self._stream()
        _check(self.lib.krig_solve(self.h, y.shape[0], y.data_ptr(), out.data_ptr()), "krig_solve")
        return out

    def solve_noalloc(self, y, out):
        """krig_solve_noalloc: the solve with the library's fixed scratch, no device allocation
        (the caller passes the output; B <= info("SOLVE_NOALLOC_MAX_B"))."""
        y = self._batch(y, (self.n,), "y", self.torch.float64)
        out = self._t(out, self.torch.float64, (y.shape[0], self.n), "out")
        self._stream()
        _check(self.lib.krig_solve_noalloc(self.h, y.shape[0], y.data_ptr(), out.data_ptr()), "krig_solve_noalloc")
        return out

    def scatter(self, alpha):
        alpha = self._batch(alpha, (self.n,), "alpha", self.torch.float64)
        out = self.empty(alpha.shape[0], self.P1, self.P2)
        self._stream()
        _check(self.lib.krig_scatter(self.h, alpha.shape[0], alpha.data_ptr(), out.data_ptr()), "krig_scatter")
        return out

    def _lag_ptr(self, lag):
        if lag is None:
            return None
        return self._t(lag, self.tdtype, (self.m1 + self.L, self.m2 + self.L), "lag").data_ptr()

    def new_saved(self, B: int):
        """Buffer for the forward row spectra kept for the adjoint (complex FP64)."""
        return self.empty(B, self.saved_per_field, 2, dtype=self.torch.float64)

    def convolve(self, alpha, lag=None, saved=None, out=None):
        alpha = self._batch(alpha, (self.n,), "alpha", self.torch.float64)
        B = alpha.shape[0]
        out = self.empty(B, self.m1, self.m2) if out is None else self._t(out, self.tdtype, (B, self.m1, self.m2), "out")
        if saved is not None:
            self._t(saved, self.torch.float64, (B, self.saved_per_field, 2), "saved")
        self._stream()
        _check(self.lib.krig_convolve(self.h, B, alpha.data_ptr(), self._lag_ptr(lag), out.data_ptr(),
                                      _ptr(saved)), "krig_convolve")
        return out

    def predict(self, y, lag=None, alpha_out=None, saved=None, out=None):
        y = self._batch(y, (self.n,), "y", self.torch.float64)
        B = y.shape[0]
        out = self.empty(B, self.m1, self.m2) if out is None else self._t(out, self.tdtype, (B, self.m1, self.m2), "out")
        if alpha_out is not None:
            self._t(alpha_out, self.torch.float64, (B, self.n), "alpha_out")
        if saved is not None:
            self._t(saved, self.torch.float64, (B, self.saved_per_field, 2), "saved")
        self._stream()
        _check(self.lib.krig_predict(self.h, B, y.data_ptr(), self._lag_ptr(lag), out.data_ptr(), _ptr(alpha_out),
                                     _ptr(saved)), "krig_predict")
        return out

    def adjoint(self, g, alpha=None, saved=None, lag=None, want_dy=True, want_dlag=True, dy_out=None,
                dlag_out=None):
        g = self._batch(g, (self.m1, self.m2), "g", self.tdtype)
        B = g.shape[0]
        if alpha is not None:
            self._t(alpha, self.torch.float64, (B, self.n), "alpha")
        if saved is not None:
            self._t(saved, self.torch.float64, (B, self.saved_per_field, 2), "saved")
        dy = None
        if want_dy:
            dy = (self.empty(B, self.n, dtype=self.torch.float64) if dy_out is None
                  else self._t(dy_out, self.torch.float64, (B, self.n), "dy_out"))
        dlag = None
        if want_dlag:
            shape = (self.m1 + self.L, self.m2 + self.L)
            dlag = self.empty(*shape) if dlag_out is None else self._t(dlag_out, self.tdtype, shape, "dlag_out")
        self._stream()
        _check(self.lib.krig_predict_adjoint(self.h, B, g.data_ptr(), _ptr(alpha), _ptr(saved), self._lag_ptr(lag),
                                             _ptr(dy), _ptr(dlag)), "krig_predict_adjoint")
        return dy, dlag

    def tune(self, key: str, value: int):
        """Set a launch shape (TUNE key): speed only, apart from DLAG_GROUP, which regroups the
        sum over fields of d lag (rounding-level change)."""
        _check(self.lib.krig_plan_tune(self.h, TUNE[key], ctypes.c_int64(int(value))), "krig_plan_tune")

    def autotune(self, B: int, with_adjoint: bool = True):
        """Time the launch-shape candidates on B synthetic fields and keep the fastest
        (krig_plan_autotune); later plans of the same shape start from the choice."""
        self._stream()
        _check(self.lib.krig_plan_autotune(self.h, int(B), 1 if with_adjoint else 0), "krig_plan_autotune")
        return {k: self.info(k) for k in ("FFT_VARIANT_ROWS", "FFT_VARIANT_COLS", "NL_ROWS64", "NL_COLS64",
                                          "DLAG_GROUP", "COLS_PAIR", "SCATTER")}

    def timing(self, on: bool):
        """Bracket every stage launch with HIP events on the plan's stream."""
        _check(self.lib.krig_timing_enable(self.h, 1 if on else 0), "krig_timing_enable")

    def timing_read(self):
        """{stage: (total_ms, launches)} since the last read (synchronises)."""
        out = {}
        for i, name in enumerate(STAGES):
            ms = ctypes.c_double()
            cnt = ctypes.c_int64()
            _check(self.lib.krig_timing_read(self.h, i, ctypes.byref(ms), ctypes.byref(cnt)), "krig_timing_read")
            out[name] = (float(ms.value), int(cnt.value))
        return out

    def predict_universal(self, z, Xs, Xg, out=None, beta_out=None, coef_out=None):
        """Universal kriging (krig_predict_universal): z [B][n] FP64, covariates Xs [np][n]
        at the sites and Xg [np][m1][m2] at the nodes (FP64) -> [B][m1][m2] (plan dtype)."""
        z = self._batch(z, (self.n,), "z", self.torch.float64)
        B = z.shape[0]
        npc = Xs.shape[0] if Xs.dim() == 2 else -1
        self._t(Xs, self.torch.float64, (npc, self.n), "Xs")
        self._t(Xg, self.torch.float64, (npc, self.m1, self.m2), "Xg")
        out = self.empty(B, self.m1, self.m2) if out is None else self._t(out, self.tdtype, (B, self.m1, self.m2), "out")
        if beta_out is not None:
            self._t(beta_out, self.torch.float64, (B, npc), "beta_out")
        if coef_out is not None:
            self._t(coef_out, self.torch.float64, (B, self.n), "coef_out")
        self._stream()
        _check(self.lib.krig_predict_universal(self.h, B, z.data_ptr(), npc, Xs.data_ptr(), Xg.data_ptr(),
                                               out.data_ptr(), _ptr(beta_out), _ptr(coef_out)),
               "krig_predict_universal")
        return out

    def interp(self, yhat, pts, q: int = 4, out=None):
        """Off-grid predictions (krig_interp): the mesh prediction yhat [B][m1][m2]
        (plan dtype) interpolated to pts [npts][2] (FP64) -> [B][npts] (plan dtype)."""
        yhat = self._batch(yhat, (self.m1, self.m2), "yhat", self.tdtype)
        B = yhat.shape[0]
        if pts.dim() != 2 or pts.shape[1] != 2:
            raise ValueError("pts: expected shape (npts, 2)")
        pts = self._t(pts, self.torch.float64, tuple(pts.shape), "pts")
        npts = pts.shape[0]
        out = self.empty(B, npts) if out is None else self._t(out, self.tdtype, (B, npts), "out")
        self._stream()
        _check(self.lib.krig_interp(self.h, B, yhat.data_ptr(), npts, pts.data_ptr(), int(q), out.data_ptr()),
               "krig_interp")
        return out

    def exact(self, alpha, out=None):
        """Exact kriging prediction on the grid (krig_predict_exact): coefficients alpha
        [B][n] FP64 -> [B][m1][m2] (plan dtype), the dense sum over the sites."""
        alpha = self._batch(alpha, (self.n,), "alpha", self.torch.float64)
        B = alpha.shape[0]
        out = self.empty(B, self.m1, self.m2) if out is None else self._t(out, self.tdtype, (B, self.m1, self.m2), "out")
        self._stream()
        _check(self.lib.krig_predict_exact(self.h, B, alpha.data_ptr(), out.data_ptr()), "krig_predict_exact")
        return out

    def exact_at(self, alpha, pts):
        """Exact kriging prediction at points (krig_exact_at): alpha [B][n] FP64,
        pts [npts][2] FP64 -> [B][npts] FP64."""
        alpha = self._batch(alpha, (self.n,), "alpha", self.torch.float64)
        B = alpha.shape[0]
        if pts.dim() != 2 or pts.shape[1] != 2:
            raise ValueError("pts: expected shape (npts, 2)")
        pts = self._t(pts, self.torch.float64, tuple(pts.shape), "pts")
        npts = pts.shape[0]
        out = self.empty(B, npts, dtype=self.torch.float64)
        self._stream()
        _check(self.lib.krig_exact_at(self.h, B, alpha.data_ptr(), npts, pts.data_ptr(), out.data_ptr()),
               "krig_exact_at")
        return out

    def kernel_at(self, i: int, pts):
        """The interpolated covariance of site i at points (krig_kernel_at): pts [npts][2]
        FP64 -> [npts] FP64."""
        if pts.dim() != 2 or pts.shape[1] != 2:
            raise ValueError("pts: expected shape (npts, 2)")
        pts = self._t(pts, self.torch.float64, tuple(pts.shape), "pts")
        out = self.empty(pts.shape[0], dtype=self.torch.float64)
        self._stream()
        _check(self.lib.krig_kernel_at(self.h, int(i), pts.shape[0], pts.data_ptr(), out.data_ptr()), "krig_kernel_at")
        return out

    def csim(self, R: int, seed: int, y):
        y = self._t(y, self.torch.float64, (self.n,), "y")
        out = self.empty(R, self.m1, self.m2)
        self._stream()
        _check(self.lib.krig_csim(self.h, R, int(seed) & 0xFFFFFFFFFFFFFFFF, y.data_ptr(), out.data_ptr()),
               "krig_csim")
        return out


def _many_args(plans, ys, outs):
    """Host arrays for the uneven-batch entry points; checks each problem's tensors."""
    if not (len(plans) == len(ys) == len(outs)) or not plans:
        raise ValueError("plans, ys and outs must be non-empty lists of equal length")
    Bs = []
    for p, y, o in zip(plans, ys, outs):
        y = p._batch(y, (p.n,), "y", p.torch.float64)
        p._t(o, p.tdtype, (y.shape[0], p.m1, p.m2), "out")
        Bs.append(y.shape[0])
    k = len(plans)
    hp = (ctypes.c_void_p * k)(*[p.h for p in plans])
    hb = (ctypes.c_int32 * k)(*Bs)
    hy = (ctypes.c_void_p * k)(*[y.data_ptr() for y in ys])
    ho = (ctypes.c_void_p * k)(*[o.data_ptr() for o in outs])
    return k, hp, hb, hy, ho


def mixture(plans, alpha, lam_sites, lam_grid, out=None):
    """Nonstationary mixture prediction (krig_mixture): plans[c] is component c's plan
    (same sites, grid and dtype); alpha [B][n] FP64, lam_sites [C][n] FP64, lam_grid
    [C][m1][m2] FP64 -> [B][m1][m2] in the plans' dtype, on torch's current stream."""
    p0 = plans[0]
    C = len(plans)
    alpha = p0._batch(alpha, (p0.n,), "alpha", p0.torch.float64)
    B = alpha.shape[0]
    p0._t(lam_sites, p0.torch.float64, (C, p0.n), "lam_sites")
    p0._t(lam_grid, p0.torch.float64, (C, p0.m1, p0.m2), "lam_grid")
    out = p0.empty(B, p0.m1, p0.m2) if out is None else p0._t(out, p0.tdtype, (B, p0.m1, p0.m2), "out")
    hp = (ctypes.c_void_p * C)(*[p.h for p in plans])
    st = p0.torch.cuda.current_stream(p0.device).cuda_stream
    _check(p0.lib.krig_mixture(hp, C, B, alpha.data_ptr(), lam_sites.data_ptr(), lam_grid.data_ptr(),
                               out.data_ptr(), st), "krig_mixture")
    return out


def predict_many(plans, ys, outs):
    """Uneven batch: plans[i].predict(ys[i], out=outs[i]) for every i, all on torch's
    current stream (krig_predict_many)."""
    k, hp, hb, hy, ho = _many_args(plans, ys, outs)
    st = plans[0].torch.cuda.current_stream(plans[0].device).cuda_stream
    _check(plans[0].lib.krig_predict_many(hp, k, hb, hy, ho, st), "krig_predict_many")
    return outs


class Batch:
    """The same uneven batch recorded once as a HIP graph (krig_batch_create) and
    replayed by launch(); ys / outs are the buffers every replay reads and writes."""

    def __init__(self, plans, ys, outs, lanes: int = 4):
        k, hp, hb, hy, ho = _many_args(plans, ys, outs)
        self.plans, self.ys, self.outs = list(plans), list(ys), list(outs)  # keep them alive
        self.lib = plans[0].lib
        self.torch = plans[0].torch
        self.device = plans[0].device
        st = self.torch.cuda.current_stream(self.device).cuda_stream
        h = ctypes.c_void_p()
        _check(self.lib.krig_batch_create(ctypes.byref(h), hp, k, hb, hy, ho, int(lanes), st), "krig_batch_create")
        self.h = h

    def launch(self):
        st = self.torch.cuda.current_stream(self.device).cuda_stream
        _check(self.lib.krig_batch_launch(self.h, st), "krig_batch_launch")
        return self.outs

    def close(self):
        if getattr(self, "h", None):
            _check(self.lib.krig_batch_destroy(self.h), "krig_batch_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_for(w, dtype: str = "f32", device: str = "cuda:0") -> Plan:
    """Plan from a workloads.Workload."""
    return Plan(w.m1, w.m2, w.x0, w.y0, w.dx, w.dy, w.L, w.sigma2, w.rho, w.nu, w.tau2, w.sites, dtype, device)


from .autograd import KrigPredictFn, krig_predict  # noqa: E402,F401
