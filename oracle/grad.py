"""Gradient of the cost (13) after unrolled iterations -- TEST INFRASTRUCTURE (only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may import it).

Two maps are differentiated, both ending in the cost (13) of the final state,

  L = sum_{f,t,m} (P / y + ln y) - 2T sum_{f,l} ln|det Q_fl|,

with every Sec. IV-A floor in place (y = max(sum_n lambda g, 1e-6), the denominators of (8)-(10)
and the IP normaliser of (16) floored at 1e-6):

* MM iterations (``mm_unrolled_*``): n iterations of eqs. (8), (9), (10) in that order with Q held
  fixed, so P = |Q x|^2 is computed once and the model variance y is refreshed after each update
  (Sec. II-B);
* full iterations (``iter_unrolled_*``): each iteration first forms the weighted covariances of
  eq. (14) from the current model and sweeps every subarray's rows in ascending order by eqs.
  (15)-(16), then computes P with the new Q and runs eqs. (8)-(10) -- the schedule of
  ``oracle.dfmnmf.iterate``.

The forward is written in PyTorch float64 on the CPU, step by step as the paper states it, and the
gradient of L with respect to the initial Q, g, W and H is PyTorch's reverse-mode differentiation
of that forward (torch.autograd), the library primitive used here; a floored quantity has zero
derivative where the floor is active.  For complex Q the gradient is dL/dRe(Q) + i dL/dIm(Q),
PyTorch's convention.
"""
from __future__ import annotations

import numpy as np
import torch

from .dfmnmf import EPS, block_offsets


def _t(a, requires_grad=False):
    t = torch.as_tensor(np.asarray(a))
    t = t.to(torch.complex128 if t.is_complex() else torch.float64)
    return t.clone().requires_grad_(requires_grad)


def powers(X, Q, mics):
    """P[f, t, o_l + mu] = |(Q_fl x^(l)_ft)_mu|^2."""
    F = X.shape[0]
    out = []
    for ml, (mo, qo) in zip(mics, block_offsets(mics)):
        Ql = Q[:, qo:qo + ml * ml].reshape(F, ml, ml)
        z = torch.einsum("fua,fta->ftu", Ql, X[:, :, mo:mo + ml])
        out.append(z.real ** 2 + z.imag ** 2)
    return torch.cat(out, dim=2)


def model(W, H, g, eps):
    """lambda[f, t, n] = sum_k W H (eq. (2)); y = max(sum_n lambda g, eps)."""
    lam = torch.einsum("nfk,nkt->ftn", W, H)
    return lam, torch.clamp(torch.einsum("ftn,fnm->ftm", lam, g), min=eps)


def update_W(W, H, g, P, eps):
    """Eq. (8): W <- W sqrt(sum_{t,m} H g P / y^2 / max(sum_{t,m} H g / y, eps))."""
    _, y = model(W, H, g, eps)
    num = torch.einsum("nkt,fnm,ftm->nfk", H, g, P / y ** 2)
    den = torch.einsum("nkt,fnm,ftm->nfk", H, g, 1.0 / y)
    return W * torch.sqrt(num / torch.clamp(den, min=eps))


def update_H(W, H, g, P, eps):
    """Eq. (9): H <- H sqrt(sum_{f,m} W g P / y^2 / max(sum_{f,m} W g / y, eps))."""
    _, y = model(W, H, g, eps)
    num = torch.einsum("nfk,fnm,ftm->nkt", W, g, P / y ** 2)
    den = torch.einsum("nfk,fnm,ftm->nkt", W, g, 1.0 / y)
    return H * torch.sqrt(num / torch.clamp(den, min=eps))


def update_g(W, H, g, P, eps):
    """Eq. (10): g <- g sqrt(sum_t lambda P / y^2 / max(sum_t lambda / y, eps))."""
    lam, y = model(W, H, g, eps)
    num = torch.einsum("ftn,ftm->fnm", lam, P / y ** 2)
    den = torch.einsum("ftn,ftm->fnm", lam, 1.0 / y)
    return g * torch.sqrt(num / torch.clamp(den, min=eps))


def cost(X, Q, g, W, H, mics, eps, P=None):
    """Eq. (13) (no additive constant); ln|det Q_f| = sum_l ln|det Q_fl|."""
    F, T, _ = X.shape
    if P is None:
        P = powers(X, Q, mics)
    _, y = model(W, H, g, eps)
    logdet = 0.0
    for ml, (_, qo) in zip(mics, block_offsets(mics)):
        logdet = logdet + torch.linalg.slogdet(Q[:, qo:qo + ml * ml].reshape(F, ml, ml))[1].sum()
    return (P / y + torch.log(y)).sum() - 2.0 * T * logdet


def mm_unrolled_cost(X, Q, g, W, H, mics, n_iter, eps=EPS):
    """The cost (13) after n_iter MM iterations (8), (9), (10) from (Q, g, W, H), Q fixed."""
    P = powers(X, Q, mics)
    for _ in range(n_iter):
        W = update_W(W, H, g, P, eps)
        H = update_H(W, H, g, P, eps)
        g = update_g(W, H, g, P, eps)
    return cost(X, Q, g, W, H, mics, eps, P=P)


def mm_unrolled_grad(X, Q, g, W, H, mics, n_iter, eps=EPS):
    """(L, dQ, dg, dW, dH) as NumPy arrays: the cost after n_iter MM iterations and its gradient with
    respect to the initial state (dQ = dL/dRe Q + i dL/dIm Q)."""
    Xt = _t(X)
    Qt, gt, Wt, Ht = (_t(a, True) for a in (Q, g, W, H))
    L = mm_unrolled_cost(Xt, Qt, gt, Wt, Ht, mics, n_iter, eps)
    grads = torch.autograd.grad(L, (Qt, gt, Wt, Ht))
    return (float(L.detach()),) + tuple(gr.detach().numpy() for gr in grads)


def mm_unrolled_state(X, Q, g, W, H, mics, n_iter, eps=EPS):
    """The state (g, W, H) after n_iter MM iterations with Q fixed (NumPy arrays)."""
    with torch.no_grad():
        Xt, Qt, gt, Wt, Ht = (_t(a) for a in (X, Q, g, W, H))
        P = powers(Xt, Qt, mics)
        for _ in range(n_iter):
            Wt = update_W(Wt, Ht, gt, P, eps)
            Ht = update_H(Wt, Ht, gt, P, eps)
            gt = update_g(Wt, Ht, gt, P, eps)
    return gt.numpy(), Wt.numpy(), Ht.numpy()


def covariances(X, y, mics):
    """Eq. (14): per subarray l, V[f, mu] = (1/T) sum_t x^(l) x^(l)H / y_{f,t,o_l+mu}."""
    T = X.shape[1]
    out = []
    for ml, (mo, _) in zip(mics, block_offsets(mics)):
        xl = X[:, :, mo:mo + ml]
        w = (1.0 / y[:, :, mo:mo + ml]).to(X.dtype)
        out.append(torch.einsum("ftu,fta,ftb->fuab", w, xl, xl.conj()) / T)
    return out


def ip_sweep(Q, V, mics, eps):
    """Eqs. (15)-(16) for every subarray, rows mu in ascending order: b = (Q_l V_mu)^-1 e_mu with
    the rows already updated, b <- b / sqrt(max(b^H V_mu b, eps)), row mu of Q_l <- b^H."""
    F = Q.shape[0]
    blocks = []
    for ml, (_, qo), Vl in zip(mics, block_offsets(mics), V):
        Ql = Q[:, qo:qo + ml * ml].reshape(F, ml, ml)
        for mu in range(ml):
            e = torch.zeros(F, ml, 1, dtype=Q.dtype)
            e[:, mu, 0] = 1.0
            b = torch.linalg.solve(Ql @ Vl[:, mu], e)[..., 0]
            s = torch.einsum("fa,fab,fb->f", b.conj(), Vl[:, mu], b).real
            b = b / torch.sqrt(torch.clamp(s, min=eps))[:, None]
            Ql = torch.cat([Ql[:, :mu], b.conj()[:, None, :], Ql[:, mu + 1:]], dim=1)
        blocks.append(Ql.reshape(F, ml * ml))
    return torch.cat(blocks, dim=1)


def iter_unrolled_cost(X, Q, g, W, H, mics, n_iter, eps=EPS):
    """The cost (13) after n_iter full iterations (eq. (14), eqs. (15)-(16), then (8)-(10))."""
    for _ in range(n_iter):
        _, y = model(W, H, g, eps)
        Q = ip_sweep(Q, covariances(X, y, mics), mics, eps)
        P = powers(X, Q, mics)
        W = update_W(W, H, g, P, eps)
        H = update_H(W, H, g, P, eps)
        g = update_g(W, H, g, P, eps)
    return cost(X, Q, g, W, H, mics, eps)


def iter_unrolled_grad(X, Q, g, W, H, mics, n_iter, eps=EPS):
    """(L, dQ, dg, dW, dH) as NumPy arrays: the cost after n_iter full iterations and its gradient
    with respect to the initial state (dQ = dL/dRe Q + i dL/dIm Q)."""
    Xt = _t(X)
    Qt, gt, Wt, Ht = (_t(a, True) for a in (Q, g, W, H))
    L = iter_unrolled_cost(Xt, Qt, gt, Wt, Ht, mics, n_iter, eps)
    grads = torch.autograd.grad(L, (Qt, gt, Wt, Ht))
    return (float(L.detach()),) + tuple(gr.detach().numpy() for gr in grads)
