"""Off-grid predictions from the mesh prediction by local polynomial interpolation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper predicts onto a regular grid only and, in its closing discussion
(Section 6), suggests reaching many irregular locations by predicting onto a
fine mesh first and then interpolating locally, for example with local
polynomials.  The reading used here:

* Interpolant: the tensor product of one-dimensional Lagrange polynomials
  through q consecutive mesh nodes in each coordinate (2 <= q <= 8), i.e. the
  unique polynomial of degree <= q-1 in x and <= q-1 in y that matches the mesh
  values on the q x q stencil.
* Stencil: for a point with t = (x - x0)/dx, i0 = floor(t) (the same FP64 rule
  as for sites), the x nodes are sx, ..., sx + q - 1 with
  sx = i0 + 1 - ceil(q/2), shifted into [0, m1 - q] at the grid edges (the
  same in y).  For even q the stencil is centred on the cell holding the point.
* Points outside the grid's bounding box have no prediction (NaN).

The Lagrange basis is written out as the textbook product
l_a(t) = prod_{k != a} (t - t_k) / (t_a - t_k).
"""
from __future__ import annotations

import math

import numpy as np

from .rapid import Grid


def stencil_start(t: float, m: int, q: int) -> int:
    """First node of the q-node stencil around grid coordinate t (0 <= t <= m-1)."""
    i0 = math.floor(t)
    return min(max(i0 + 1 - (q + 1) // 2, 0), m - q)


def lagrange_weights(t: float, nodes: np.ndarray) -> np.ndarray:
    """Values at t of the Lagrange basis polynomials through the given nodes."""
    q = len(nodes)
    w = np.ones(q)
    for a in range(q):
        for k in range(q):
            if k != a:
                w[a] *= (t - nodes[k]) / (nodes[a] - nodes[k])
    return w


def interp_points(g: Grid, yhat: np.ndarray, pts: np.ndarray, q: int) -> np.ndarray:
    """Off-grid predictions at pts (n x 2) from the mesh prediction yhat (m1 x m2),
    one point at a time (pure Python loops: small cases only)."""
    yhat = np.asarray(yhat, dtype=np.float64)
    out = np.empty(len(pts))
    for j, (x, y) in enumerate(np.asarray(pts, dtype=np.float64)):
        t = (x - g.x0) / g.dx
        u = (y - g.y0) / g.dy
        if not (0.0 <= t <= g.m1 - 1 and 0.0 <= u <= g.m2 - 1):
            out[j] = np.nan
            continue
        sx = stencil_start(t, g.m1, q)
        sy = stencil_start(u, g.m2, q)
        wx = lagrange_weights(t, np.arange(sx, sx + q, dtype=np.float64))
        wy = lagrange_weights(u, np.arange(sy, sy + q, dtype=np.float64))
        out[j] = wx @ yhat[sx:sx + q, sy:sy + q] @ wy
    return out
