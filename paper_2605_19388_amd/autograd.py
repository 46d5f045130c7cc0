"""torch.autograd.Function over the library's unrolled-MM gradient.

``unrolled_mm_cost(X, Q, g, W, H, mics, n_iter)`` returns the cost (13) after n_iter MM
iterations of eqs. (8), (9), (10) (Q held fixed) from the state (Q, g, W, H), as a 0-d float64
tensor; its backward is the library's hand-written reverse pass (dfm_mm_backward), whose forward
iterations stored per-iteration checkpoints.  Argument marshalling only: both passes run in the
HIP kernels of libdfmnmf.so.
"""
from __future__ import annotations

import torch

from .binding import DistributedFastMNMF


class UnrolledMMCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, Q, g, W, H, mics, n_iter, eps):
        N, _, K = W.shape
        p = DistributedFastMNMF(X.detach(), mics, N, K, W=W.detach(), H=H.detach(), Q=Q.detach(), g=g.detach(),
                                eps=eps, device=X.device)
        tape = p.mm_forward(n_iter)
        cost = p.nll()
        ctx.plan, ctx.tape = p, tape
        return torch.tensor(cost, dtype=torch.float64, device=X.device)

    @staticmethod
    def backward(ctx, grad_out):
        dQ, dg, dW, dH = ctx.plan.mm_backward(ctx.tape)
        s = grad_out.to(dg.dtype)
        return None, dQ * s, dg * s, dW * s, dH * s, None, None, None


def unrolled_mm_cost(X, Q, g, W, H, mics, n_iter, eps=1e-6):
    return UnrolledMMCost.apply(X, Q, g, W, H, tuple(int(m) for m in mics), int(n_iter), float(eps))
