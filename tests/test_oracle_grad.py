"""Pins of the oracle's gradient of the cost after unrolled iterations (oracle/grad.py) -- CPU
only.  MM iterations (Q fixed) and full iterations (eq. (14), the IP sweep of eqs. (15)-(16), then
eqs. (8)-(10)):

* its forward equals the NumPy oracle's updates and cost (two independent writings; for full
  iterations, ``oracle.dfmnmf.iterate`` with its own solves);
* its gradient equals FP64 central finite differences (step 1e-6) of the NumPy oracle, for every
  parameter block and the real and imaginary parts of Q, with and without floors active;
* at an MM fixed point (a recording with |Q x|^2 = y exactly) the gradient with respect to g, W
  and H is zero, for the cost itself and after any number of unrolled iterations (the MM updates
  are the identity there and their outputs' adjoints vanish);
* with no iteration, dL/dW = den_W - num_W of eq. (8) (the MM terms are the cost's gradient).
"""
import numpy as np
import pytest

from oracle import dfmnmf as D
from oracle import grad as G
from tests.common import random_state
from paper_2605_19388_amd import synth


def _case(F=2, T=6, mics=(2, 1), N=2, K=2, seed=3, scale=1.0):
    X = scale * synth.mixture(F, T, mics, N, K, seed)
    Q, g, W, H = random_state(F, T, mics, N, K, seed + 1)
    return X, Q, g, W, H


def _numpy_unrolled_cost(X, Q, g, W, H, mics, n_iter):
    P = D.powers(X, Q, mics)
    for _ in range(n_iter):
        W = D.update_W(W, H, g, P)
        H = D.update_H(W, H, g, P)
        g = D.update_g(W, H, g, P)
    return D.nll(X, Q, g, W, H, mics)


def test_forward_equals_numpy_oracle():
    X, Q, g, W, H = _case(F=4, T=20, mics=(2, 2), N=3, K=3)
    mics = (2, 2)
    gn, Wn, Hn = G.mm_unrolled_state(X, Q, g, W, H, mics, 3)
    P = D.powers(X, Q, mics)
    for _ in range(3):
        W = D.update_W(W, H, g, P)
        H = D.update_H(W, H, g, P)
        g = D.update_g(W, H, g, P)
    np.testing.assert_allclose(gn, g, rtol=1e-12)
    np.testing.assert_allclose(Wn, W, rtol=1e-12)
    np.testing.assert_allclose(Hn, H, rtol=1e-12)
    L, *_ = G.mm_unrolled_grad(X, Q, *(a for a in (g, W, H)), mics, 0)
    assert abs(L - D.nll(X, Q, g, W, H, mics)) <= 1e-12 * abs(L)


def _numpy_iter_cost(X, Q, g, W, H, mics, n_iter):
    return D.nll(X, *D.iterate(X, Q, g, W, H, mics, n_iter), mics)


def _fd_check(X, Q, g, W, H, mics, n_iter, samples=6, seed=0, rtol=1e-5, full=False):
    grad_fn, cost_fn = (G.iter_unrolled_grad, _numpy_iter_cost) if full else (G.mm_unrolled_grad, _numpy_unrolled_cost)
    L, dQ, dg, dW, dH = grad_fn(X, Q, g, W, H, mics, n_iter)
    rng = np.random.Generator(np.random.PCG64(seed))
    params = {"Q": Q, "g": g, "W": W, "H": H}
    grads = {"Q": dQ, "g": dg, "W": dW, "H": dH}
    scale = max(abs(L), 1.0)
    for name, p in params.items():
        for _ in range(samples):
            idx = tuple(int(rng.integers(0, s)) for s in p.shape)
            parts = [(1.0, "re"), (1j, "im")] if np.iscomplexobj(p) else [(1.0, "re")]
            for unit, part in parts:
                h = 1e-6 * (abs(p[idx]) if p[idx] != 0 else 1.0)  # step 1e-6 relative to the entry
                args = {k: v.copy() for k, v in params.items()}
                args[name][idx] += unit * h
                lp = cost_fn(X, args["Q"], args["g"], args["W"], args["H"], mics, n_iter)
                args[name][idx] -= 2 * unit * h
                lm = cost_fn(X, args["Q"], args["g"], args["W"], args["H"], mics, n_iter)
                fd = (lp - lm) / (2 * h)
                got = grads[name][idx].real if part == "re" else grads[name][idx].imag
                noise = 64 * np.finfo(float).eps * scale / h  # rounding of the two costs, over the step
                assert abs(got - fd) <= rtol * max(abs(fd), 1e-3 * scale / p.size) + noise, (name, idx, part, got, fd)


@pytest.mark.parametrize("n_iter", [0, 1, 3])
def test_gradient_equals_central_finite_differences(n_iter):
    X, Q, g, W, H = _case()
    _fd_check(X, Q, g, W, H, (2, 1), n_iter)


def test_gradient_equals_finite_differences_with_floors_active():
    """A faint recording with a small model: y floored at some bins, the g denominators floored."""
    X, Q, g, W, H = _case(scale=1e-3)
    W, H = 3e-4 * W, 3e-4 * H
    y = D.model_variance(D.source_psd(W, H), g)
    assert np.any(y == D.EPS) and np.any(y > D.EPS)
    _fd_check(X, Q, g, W, H, (2, 1), 2, seed=1)


def _fixed_point_case(F=3, T=8, mics=(2, 2), N=2, K=2, seed=9):
    """Q = I and x_ftm = sqrt(y_ftm) e^{i phi}: P = y, so every MM update is the identity."""
    _, g, W, H = random_state(F, T, mics, N, K, seed)
    Q = synth.initial_state(F, T, mics, N, K, seed)[0]
    y = D.model_variance(D.source_psd(W, H), g)
    rng = np.random.Generator(np.random.PCG64(seed))
    X = np.sqrt(y) * np.exp(2j * np.pi * rng.random(y.shape))
    return X, Q, g, W, H, mics


@pytest.mark.parametrize("n_iter", [0, 2])
def test_gradient_vanishes_at_an_mm_fixed_point(n_iter):
    X, Q, g, W, H, mics = _fixed_point_case()
    np.testing.assert_allclose(D.update_W(W, H, g, D.powers(X, Q, mics)), W, rtol=1e-12)
    L, dQ, dg, dW, dH = G.mm_unrolled_grad(X, Q, g, W, H, mics, n_iter)
    for name, d, p in (("g", dg, g), ("W", dW, W), ("H", dH, H)):
        assert np.abs(d * p).max() <= 1e-10 * abs(L), name   # relative to the cost's scale


def test_direct_gradient_is_den_minus_num():
    X, Q, g, W, H = _case(F=3, T=10, mics=(2, 2), N=2, K=3)
    mics = (2, 2)
    _, _, dg, dW, dH = G.mm_unrolled_grad(X, Q, g, W, H, mics, 0)
    P = D.powers(X, Q, mics)
    for d, terms in ((dW, D.mm_terms_W), (dH, D.mm_terms_H), (dg, D.mm_terms_g)):
        num, den = terms(W, H, g, P)
        np.testing.assert_allclose(d, den - num, rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------- full iterations (IP sweep + MM)
@pytest.mark.parametrize("mics", [(2, 1), (2, 2), (1, 1, 2)])
def test_iter_forward_equals_numpy_oracle(mics):
    X, Q, g, W, H = _case(F=3, T=12, mics=mics, N=2, K=2)
    for n_iter in (0, 1, 3):
        L, *_ = G.iter_unrolled_grad(X, Q, g, W, H, mics, n_iter)
        ref = _numpy_iter_cost(X, Q, g, W, H, mics, n_iter)
        assert abs(L - ref) <= 1e-12 * abs(ref), (n_iter, L, ref)


@pytest.mark.parametrize("n_iter", [1, 2])
def test_iter_gradient_equals_central_finite_differences(n_iter):
    X, Q, g, W, H = _case()
    _fd_check(X, Q, g, W, H, (2, 1), n_iter, full=True)


def test_iter_gradient_equals_finite_differences_with_floors_active():
    """Floors of y and of the MM denominators active (a faint recording, a small model)."""
    X, Q, g, W, H = _case(scale=1e-3)
    W, H = 3e-4 * W, 3e-4 * H
    y = D.model_variance(D.source_psd(W, H), g)
    assert np.any(y == D.EPS) and np.any(y > D.EPS)
    _fd_check(X, Q, g, W, H, (2, 1), 1, seed=2, full=True)


def test_iter_gradient_with_the_normaliser_floor_active():
    """A loud recording with a model that keeps y unfloored: V is so large that b^H V b < 1e-6 for
    every first row of the sweep, so the normaliser of eq. (16) is floored there.  The forward
    still equals the NumPy oracle's (whose floor is pinned on its own) and the gradient its central
    differences (the floored normaliser has zero derivative)."""
    mics = (2, 1)
    X, Q, g, W, H = _case(F=3, T=12, mics=mics, N=2, K=2, scale=1e5)
    W, H = 1e-3 * W, 1e-3 * H
    y = D.model_variance(D.source_psd(W, H), g)
    assert np.all(y > D.EPS)
    V = D.weighted_covariances(X, y, mics)
    s = [float((b.conj() @ Vl[f, 0] @ b).real)
         for Ql, Vl, ml in zip(D.q_blocks(Q, mics), V, mics) for f in range(3)
         for b in [np.linalg.solve(Ql[f] @ Vl[f, 0], np.eye(ml)[:, 0])]]
    assert max(s) < D.EPS
    L, *_ = G.iter_unrolled_grad(X, Q, g, W, H, mics, 1)
    ref = _numpy_iter_cost(X, Q, g, W, H, mics, 1)
    assert abs(L - ref) <= 1e-12 * abs(ref)
    _fd_check(X, Q, g, W, H, mics, 1, seed=4, full=True)


@pytest.mark.parametrize("mics", [(2, 1), (3, 2)])
def test_iter_gradient_vanishes_on_rows_the_sweep_overwrites_first(mics):
    """The sweep replaces row 1 of each block by a vector fixed, up to its phase, by the other rows
    alone (Q V b = e_1 fixes b's direction through the other rows' equations; the scale is then
    normalised away), and the cost ignores row phases; so after a full iteration the cost does not
    depend on the first row of any block, and its gradient there is exactly zero."""
    X, Q, g, W, H = _case(F=3, T=12, mics=mics, N=2, K=2)
    L, dQ, *_ = G.iter_unrolled_grad(X, Q, g, W, H, mics, 1)
    blocks = D.q_blocks(dQ, mics)
    top = max(np.abs(b).max() for b in blocks)
    for b in blocks:
        assert np.abs(b[:, 0, :]).max() <= 1e-12 * top
    assert max(np.abs(b[:, 1:, :]).max() for b in blocks if b.shape[1] > 1) > 1e-3 * top


def test_iter_gradient_without_iterations_is_the_cost_gradient():
    X, Q, g, W, H = _case(F=3, T=10, mics=(2, 2), N=2, K=3)
    a = G.iter_unrolled_grad(X, Q, g, W, H, (2, 2), 0)
    b = G.mm_unrolled_grad(X, Q, g, W, H, (2, 2), 0)
    for u, v in zip(a[1:], b[1:]):
        np.testing.assert_allclose(u, v, rtol=1e-13, atol=1e-15)
