"""Gradients of the rapid predictor (the adjoint of eqs. ApproxPrediction2/Convolution).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The forward map is
    c = M^{-1} y                (eq. findc),
    c* = A^T c                  (Step 5),
    y_hat[a, b] = sum_{p,q} lag[|a+L-p|, |b+L-q|] c*[p, q]   (eq. Convolution,
                                                              unpadded outputs).
For an upstream gradient g = d loss / d y_hat (m1 x m2) the chain rule gives
    d loss / d c*[p, q] = sum_{a,b} g[a, b] lag[|a+L-p|, |b+L-q|]     (corr image)
    d loss / d c       = A vec(d loss / d c*)
    d loss / d y       = M^{-1} d loss / d c        (M symmetric)
    d loss / d lag[u, w] = sum over (a, b, p, q) with |a+L-p| = u, |b+L-q| = w
                           of g[a, b] c*[p, q].
A and c are held fixed with respect to the lag image (the interpolation kernel
and the prediction kernel may differ, as the discussion of nonstationary
extensions notes).  Everything below is the direct O(N * nnz) definition.
"""
from __future__ import annotations

import numpy as np

from .rapid import Grid


def corr_image_direct(grid: Grid, lag: np.ndarray, g: np.ndarray) -> np.ndarray:
    """d loss / d c* over the padded P1 x P2 grid by direct summation."""
    g = np.asarray(g, dtype=np.float64)
    out = np.zeros((grid.P1, grid.P2))
    a = np.arange(grid.m1)
    b = np.arange(grid.m2)
    for p in range(grid.P1):
        du = np.abs(a + grid.L - p)                        # m1
        for q in range(grid.P2):
            dw = np.abs(b + grid.L - q)                    # m2
            out[p, q] = np.sum(g * lag[np.ix_(du, dw)])
    return out


def grad_coef(A, corr: np.ndarray) -> np.ndarray:
    """d loss / d c = A vec(corr)."""
    return A @ np.asarray(corr, dtype=np.float64).ravel()


def dlag_direct(grid: Grid, g: np.ndarray, cimg: np.ndarray) -> np.ndarray:
    """d loss / d lag over the (m1+L) x (m2+L) quadrant by direct summation."""
    g = np.asarray(g, dtype=np.float64)
    cimg = np.asarray(cimg, dtype=np.float64)
    out = np.zeros((grid.m1 + grid.L, grid.m2 + grid.L))
    pp, qq = np.nonzero(cimg)
    a = np.arange(grid.m1)
    b = np.arange(grid.m2)
    for p, q in zip(pp, qq):
        du = np.abs(a + grid.L - p)
        dw = np.abs(b + grid.L - q)
        np.add.at(out, (du[:, None], dw[None, :]), g * cimg[p, q])
    return out


def dlag_entry(grid: Grid, g: np.ndarray, cimg: np.ndarray, u: int, w: int) -> float:
    """One entry of d loss / d lag: sum over the sign images (+-u, +-w).

    A lag of 0 in either coordinate has a single sign image.
    """
    g = np.asarray(g, dtype=np.float64)
    tot = 0.0
    su = (u,) if u == 0 else (u, -u)
    sw = (w,) if w == 0 else (w, -w)
    for du in su:
        for dw in sw:
            # output (a, b) pairs with source (p, q) = (a + L - du, b + L - dw)
            for a in range(grid.m1):
                p = a + grid.L - du
                if p < 0 or p >= grid.P1:
                    continue
                qs = np.arange(grid.m2) + grid.L - dw
                ok = (qs >= 0) & (qs < grid.P2)
                tot += float(np.sum(g[a, ok] * cimg[p, qs[ok]]))
    return tot


def loss_masked_square(yhat: np.ndarray, mask: np.ndarray) -> float:
    """The differentiation workload's loss: sum over the grid of m * y_hat^2."""
    return float(np.sum(mask * yhat * yhat))


def corr_image_fft(grid: Grid, lag: np.ndarray, g: np.ndarray) -> np.ndarray:
    """TEST-ONLY FFT form of corr_image_direct (validated against it in the test suite)."""
    from .rapid import embed_even, fft_len
    F1 = fft_len(grid.m1 + grid.P1 - 1)
    F2 = fft_len(grid.m2 + grid.P2 - 1)
    E = embed_even(lag, F1, F2)
    G = np.zeros((F1, F2))
    G[grid.L:grid.L + grid.m1, grid.L:grid.L + grid.m2] = g
    return np.fft.ifft2(np.fft.fft2(E) * np.fft.fft2(G)).real[:grid.P1, :grid.P2]


def dlag_fft(grid: Grid, g: np.ndarray, cimg: np.ndarray) -> np.ndarray:
    """TEST-ONLY FFT form of dlag_direct: fold of the cross-correlation of g (at offset L)
    with c*, X[d] = sum_p g_pad[p] c*[p - d], over the sign images (validated against
    dlag_direct in the test suite)."""
    from .rapid import fft_len
    F1 = fft_len(grid.m1 + grid.P1 - 1)
    F2 = fft_len(grid.m2 + grid.P2 - 1)
    G = np.zeros((F1, F2))
    G[grid.L:grid.L + grid.m1, grid.L:grid.L + grid.m2] = g
    C = np.zeros((F1, F2))
    C[:grid.P1, :grid.P2] = cimg
    X = np.fft.ifft2(np.fft.fft2(G) * np.conj(np.fft.fft2(C))).real
    n1, n2 = grid.m1 + grid.L, grid.m2 + grid.L
    out = np.zeros((n1, n2))
    for u in range(n1):
        rows = [u] if u == 0 else [u, F1 - u]
        for w in range(n2):
            cols = [w] if w == 0 else [w, F2 - w]
            out[u, w] = sum(X[r, c] for r in rows for c in cols)
    return out
