"""torch.autograd.Function over the 2-pass randomized Cholesky QR.

forward:  (Q, R) = RCholQR2(X) on the GPU (Algorithm 3); saves X, R_s and
          R' -- not Q, which backward recomputes with the forward kernels.
backward: dX = (dQ + Q copyltu(R dR^T - dQ^T Q)) R^{-T} in librcholqr.
"""
import torch

from . import binding as _b


class RCholQR2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, k, seed, kind=_b.GAUSSIAN, precision=None):
        Q, R, ex = _b.factor(X.detach(), k, seed, kind, 2, precision, want_factors=True)
        ctx.save_for_backward(X.detach(), ex["Rs"], ex["Rp"])
        ctx.precision = precision
        ctx.mark_non_differentiable()
        return Q, R

    @staticmethod
    def backward(ctx, dQ, dR):
        X, Rs, Rp = ctx.saved_tensors
        if dQ is None:
            dQ = torch.zeros_like(X)
        dX = _b.backward(X, Rs, Rp, dQ.to(X.dtype), dR, ctx.precision)
        return dX, None, None, None, None


def rcholqr2(X, k, seed, kind=_b.GAUSSIAN, precision=None):
    """Differentiable 2-pass factorisation: returns (Q, R)."""
    return RCholQR2.apply(X, k, seed, kind, precision)
