"""torch.autograd.Function over the library's unrolled-iteration gradients.

``unrolled_mm_cost(X, Q, g, W, H, mics, n_iter)`` returns the cost (13) after n_iter MM
iterations of eqs. (8), (9), (10) (Q held fixed) from the state (Q, g, W, H), as a 0-d float64
tensor; its backward is the library's hand-written reverse pass (dfm_mm_backward), whose forward
iterations stored per-iteration checkpoints.  ``unrolled_iter_cost`` is the same over full
iterations (eq. (14), the IP sweep (15)-(16), then (8)-(10); dfm_iter_forward / dfm_iter_backward).
Argument marshalling only: both passes run in the HIP kernels of libdfmnmf.so.
"""
from __future__ import annotations

import torch

from .binding import DistributedFastMNMF


class UnrolledCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, Q, g, W, H, mics, n_iter, eps, kind):
        N, _, K = W.shape
        p = DistributedFastMNMF(X.detach(), mics, N, K, W=W.detach(), H=H.detach(), Q=Q.detach(), g=g.detach(),
                                eps=eps, device=X.device)
        tape = getattr(p, f"{kind}_forward")(n_iter)
        cost = p.nll()
        ctx.plan, ctx.tape, ctx.kind = p, tape, kind
        return torch.tensor(cost, dtype=torch.float64, device=X.device)

    @staticmethod
    def backward(ctx, grad_out):
        dQ, dg, dW, dH = getattr(ctx.plan, f"{ctx.kind}_backward")(ctx.tape)
        s = grad_out.to(dg.dtype)
        return None, dQ * s, dg * s, dW * s, dH * s, None, None, None, None


def unrolled_mm_cost(X, Q, g, W, H, mics, n_iter, eps=1e-6):
    return UnrolledCost.apply(X, Q, g, W, H, tuple(int(m) for m in mics), int(n_iter), float(eps), "mm")


def unrolled_iter_cost(X, Q, g, W, H, mics, n_iter, eps=1e-6):
    return UnrolledCost.apply(X, Q, g, W, H, tuple(int(m) for m in mics), int(n_iter), float(eps), "iter")
