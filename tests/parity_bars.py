"""Parity bars shared by the GPU tests: relative max error per field against the FP64 oracle.

- FP64 plans: 1e-12 where both sides compute from identical inputs (the FP64 target).  A case
  that FP64 rounding of a cancellation-heavy sum (sum |c*| / max |y_hat| up to ~1e5) puts above
  it is named in FP64_EXCEPTIONS with its measured error and cancellation and held to a bar of its
  own; no bar is scaled by a formula.
- FP32 plans compute in FP64 but read and write FP32 caller arrays (lag, upstream gradient,
  predictions, lag gradient) and store three intermediate spectra in FP32: predictions and the
  lag gradient are held to 1e-5 (the FP32 target), dy (an FP64 output whose FP32 inputs move it by
  ~1e-7) to 1e-6.
Each check prints the case, the error and the bar it was held to.
"""
BAR_F64 = 1e-12
BAR_F32 = 1e-5
BAR_F32_DY = 1e-6

# case label -> (bar, measured error, cancellation) for FP64 cases above BAR_F64: the longest
# transforms of the sweep (a 1500 x 12 grid, column length 3072) with the largest cancellation
FP64_EXCEPTIONS = {
    "sweep 1500x12 L2 n80 field 0": (2e-12, 1.35e-12, 5.7e4),
    "sweep 1500x12 L2 n80 field 1": (2e-12, None, 5.6e4),
}


def bar_for(dtype, label=None):
    if dtype == "f32":
        return BAR_F32
    if label is not None and label in FP64_EXCEPTIONS:
        return FP64_EXCEPTIONS[label][0]
    return BAR_F64


def check(label, err, bar, extra=""):
    print(f"[parity] {label}: err {err:.3e} bar {bar:.1e} {extra}".rstrip(), flush=True)
    assert err < bar, (label, err, bar, extra)


def check_all(items):
    """check() every (label, err, bar, extra) item, printing all of them before failing."""
    failed = []
    for item in items:
        try:
            check(*item)
        except AssertionError as e:
            failed.append(e.args[0])
    assert not failed, failed


def weight_residual_ratio(W, KN, kv):
    """max over sites of |K_N w_i - k_i|_inf / (10 M eps |K_N|_inf |w_i|_inf): the residual of
    eq. weights against the bound of a backward-stable solve (below 1 passes)."""
    import numpy as np
    res = np.abs(W @ KN - kv).max(axis=1)
    bound = 10 * KN.shape[0] * np.finfo(float).eps * np.abs(KN).sum(axis=1).max() * np.abs(W).max(axis=1)
    return float((res / bound).max())
