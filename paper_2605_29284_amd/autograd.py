"""torch.autograd.Function around the rapid predictor and its hand-written adjoint.

forward(y, lag) -> y_hat    (krig_predict; saves alpha and the row spectra of c*)
backward(g)     -> (dy, dlag) (krig_predict_adjoint)

dy = (K + tau^2 I)^{-1} A corr(Phi, g) is the gradient w.r.t. the data, dlag the
gradient w.r.t. the lag image (so covariance parameters can be trained through a
lag image built from them); the interpolation weights A and the kriging factor
are constants of the plan.
"""
from __future__ import annotations

import torch


class KrigPredictFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, y, lag=None):
        yb = y.detach()
        squeeze = yb.dim() == 1
        if squeeze:
            yb = yb.unsqueeze(0)
        yb = yb.contiguous()
        B = yb.shape[0]
        alpha = torch.empty(B, plan.n, dtype=torch.float64, device=yb.device)
        saved = plan.new_saved(B)
        lag_d = None if lag is None else lag.detach().contiguous()
        out = plan.predict(yb, lag=lag_d, alpha_out=alpha, saved=saved)
        ctx.plan = plan
        ctx.squeeze = squeeze
        ctx.has_lag = lag is not None
        ctx.save_for_backward(alpha, saved, lag_d if lag_d is not None else torch.empty(0))
        return out[0] if squeeze else out

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        alpha, saved, lag_d = ctx.saved_tensors
        gb = g.unsqueeze(0) if ctx.squeeze else g
        gb = gb.to(plan.tdtype).contiguous()
        want_dy = ctx.needs_input_grad[1]
        want_dlag = ctx.has_lag and ctx.needs_input_grad[2]
        dy, dlag = plan.adjoint(gb, alpha=alpha, saved=saved, lag=lag_d if ctx.has_lag else None,
                                want_dy=want_dy, want_dlag=want_dlag)
        if dy is not None and ctx.squeeze:
            dy = dy[0]
        return None, dy, dlag


def krig_predict(plan, y, lag=None):
    """Differentiable rapid prediction (see KrigPredictFn)."""
    return KrigPredictFn.apply(plan, y, lag)
