"""Pins of the oracle's 1e-6 floors (Sec. IV-A) with the floors active (CPU only).

Sec. IV-A floors three quantities at 1e-6: the model variance eta (y here), the
denominators of the MM updates (8)-(10), and the normaliser of (7)/(16).  The
configurations elsewhere keep every floor inactive, so these cases are built so
that each floor decides the result, and each case first asserts that the floor
it pins is active (a pin of an inactive floor would pass with any floor):

* tiny NMF parameters (W, H ~ 1e-15) and a faint recording (X ~ 1e-6): the
  model variance is floored at every (f, t, m) and every MM denominator lies
  below 1e-6;
* a loud recording (X ~ 1e6) with an ordinary model: every IP normaliser
  b^H V b lies below 1e-6.

Each case is checked against what the floors fix independently of the
oracle's code:

* conventional FastMNMF (Sec. II-A, eqs. (4)-(10)), written separately in the
  paper's notation with its own floors, which distributed FastMNMF with one
  subarray must equal stage by stage (Sec. III-B, end);
* closed forms: with eta floored everywhere, every V_mu of eq. (14) is the
  same matrix R / 1e-6 (R the sample covariance), so the first sweep whitens:
  Q R Q^H = 1e-6 I; with a single mic and a floored normaliser, the row is
  1 / (conj(q) v sqrt(1e-6)) instead of phase(q) / sqrt(v); with eta floored
  everywhere the model is the Gaussian of eq. (1) with the fixed covariance
  1e-6 (Q^H Q)^{-1}, whose likelihood is computed by brute force.

``check_*`` functions take the oracle module as an argument so that
tests/test_oracle_mutations.py can run them against copies of the oracle with
mistakes planted in their floors.
"""
import numpy as np
import pytest

from oracle import conventional, dfmnmf as D, fullcov
from paper_2605_19388_amd import synth
from tests.common import random_state, rel

EPS = 1e-6  # the floor of Sec. IV-A


def faint_case(mics=(3,), F=3, T=12, N=2, K=2, seed=71):
    """Model floored everywhere: W, H ~ 1e-15 (so sum_n lambda g ~ 1e-28), X ~ 1e-6."""
    X = 1e-6 * synth.mixture(F, T, mics, N, K, seed=seed)
    Q, g, W, H = random_state(F, T, mics, N, K, seed=seed + 1)
    return X, Q, g, 1e-15 * W, 1e-15 * H


def loud_case(mics=(3,), F=3, T=12, N=2, K=2, seed=81):
    """Ordinary model (y ~ 1), loud recording X ~ 1e6: V >~ 1e9 (sensor noise 1e-3 included), so b^H V b <~ 1e-9."""
    X = 1e6 * synth.mixture(F, T, mics, N, K, seed=seed)
    Q, g, W, H = random_state(F, T, mics, N, K, seed=seed + 1)
    return X, Q, g, W, H


def _raw_model(W, H, g):
    """sum_n lambda_ftn g_fnm without any floor, by explicit loops over n and k (eq. (2))."""
    lam = fullcov.source_spectrogram(W, H)                     # [F, T, N]
    F, T, N = lam.shape
    M = g.shape[2]
    y = np.zeros((F, T, M))
    for n in range(N):
        y += lam[:, :, n, None] * g[:, None, n, :]
    return y


def _conv(X, Q, g, W, H, mics):
    Wt = np.conj(np.transpose(fullcov.blockdiag_transform(D.q_blocks(Q, mics)), (0, 2, 1)))
    return conventional.FastMNMF(X, Wt, np.transpose(W, (1, 2, 0)), np.transpose(H, (1, 2, 0)), g, floor=EPS)


# ----------------------------------------------------------------- checks (module under test as argument)
def check_floored_stages_equal_conventional(Dm, case):
    """Every stage of two iterations with one subarray equals conventional FastMNMF with its own floors."""
    mics = (3,)
    X, Q, g, W, H = case(mics)
    F = X.shape[0]
    conv = _conv(X, Q, g, W, H, mics)
    stages = []
    Dm.iterate(X, Q, g, W, H, mics, 2,
               callback=lambda s, Q, g, W, H: stages.append((s, Q.copy(), g.copy(), W.copy(), H.copy())))
    steps = [conv.update_W, conv.update_t, conv.update_v, conv.update_lam] * 2
    assert len(stages) == len(steps)
    for (stage, Qs, gs, Ws, Hs), step in zip(stages, steps):
        step()
        assert rel(Qs.reshape(F, 3, 3), np.conj(np.transpose(conv.Wt, (0, 2, 1)))) < 1e-10, stage
        assert rel(Ws, np.transpose(conv.t, (2, 0, 1))) < 1e-10, stage
        assert rel(Hs, np.transpose(conv.v, (2, 0, 1))) < 1e-10, stage
        assert rel(gs, conv.lam) < 1e-10, stage
        c = conv.cost()
        assert abs(Dm.nll(X, Qs, gs, Ws, Hs, mics) - c) < 1e-10 * abs(c), stage


def check_floored_model_whitens(Dm):
    """eta floored everywhere => V_mu = R / 1e-6 for every mu => one sweep gives Q R Q^H = 1e-6 I."""
    mics = (2, 3)
    X, Q, g, W, H = faint_case(mics)
    T = X.shape[1]
    y = Dm.model_variance(Dm.source_psd(W, H), g)
    Q2 = Dm.q_blocks(Dm.ip_sweep(Q, Dm.weighted_covariances(X, y, mics), mics), mics)
    for l, (mo, _) in enumerate(Dm.block_offsets(mics)):
        xl = X[:, :, mo:mo + mics[l]]
        R = np.einsum("fta,ftb->fab", xl, xl.conj()) / T
        QRQ = np.einsum("fab,fbc,fdc->fad", Q2[l], R, Q2[l].conj())
        np.testing.assert_allclose(QRQ / EPS, np.broadcast_to(np.eye(mics[l]), QRQ.shape), atol=1e-9)


def check_floored_model_likelihood(Dm):
    """eta floored everywhere => eq. (13) is the brute-force Gaussian likelihood of eq. (1) with the fixed
    block-diagonal covariance 1e-6 (Q^H Q)^{-1}: sum_ft [x^H S^-1 x + ln det S]."""
    mics = (2, 1)
    X, Q, g, W, H = faint_case(mics, F=2, T=9)
    F, T, M = X.shape
    Qf = fullcov.blockdiag_transform(D.q_blocks(Q, mics))
    ref = 0.0
    for f in range(F):
        S = EPS * np.linalg.inv(Qf[f].conj().T @ Qf[f])
        for t in range(T):
            ref += float(np.real(X[f, t].conj() @ np.linalg.solve(S, X[f, t]))) + np.linalg.slogdet(S)[1]
    got = Dm.nll(X, Q, g, W, H, mics)
    assert abs(got - ref) <= 1e-10 * abs(ref), (got, ref)


def check_floored_normaliser_single_mic(Dm):
    """M_l = 1 with |q|^2 v > 1e6: b^H V b = 1 / (|q|^2 v) < 1e-6 is floored, so the new row is
    conj(b) / sqrt(1e-6) = 1 / (conj(q) v sqrt(1e-6)) (eqs. (15)-(16))."""
    mics = (1, 1)
    X, Q, g, W, H = loud_case(mics, F=4, T=20)
    y = Dm.model_variance(Dm.source_psd(W, H), g)
    V = Dm.weighted_covariances(X, y, mics)
    Q2 = Dm.ip_sweep(Q, V, mics)
    for m in range(2):
        v = V[m][:, 0, 0, 0].real
        q = Q[:, m]
        assert np.all(np.abs(q) ** 2 * v > 1.0 / EPS)
        np.testing.assert_allclose(Q2[:, m], 1.0 / (np.conj(q) * v * np.sqrt(EPS)), rtol=1e-12)


def check_floored_mm_closed_form(Dm):
    """eta floored everywhere and den < 1e-6: the MM updates (8)-(10) become
    theta * sqrt(num / 1e-6) with num = sum (weights) P / 1e-12, written here as explicit loops."""
    mics = (2, 2)
    X, Q, g, W, H = faint_case(mics, F=2, T=6, N=2, K=2)
    F, T, M = X.shape
    N, _, K = W.shape
    P = Dm.powers(X, Q, mics)
    W1 = Dm.update_W(W, H, g, P)
    for n in range(N):
        for f in range(F):
            for k in range(K):
                num = sum(H[n, k, t] * g[f, n, m] * P[f, t, m] for t in range(T) for m in range(M)) / EPS ** 2
                den = sum(H[n, k, t] * g[f, n, m] for t in range(T) for m in range(M)) / EPS
                assert den < EPS
                assert abs(W1[n, f, k] - W[n, f, k] * np.sqrt(num / EPS)) <= 1e-12 * W1[n, f, k]
    H1 = Dm.update_H(W1, H, g, P)
    for n in range(N):
        for k in range(K):
            for t in range(T):
                num = sum(W1[n, f, k] * g[f, n, m] * P[f, t, m] for f in range(F) for m in range(M)) / EPS ** 2
                den = sum(W1[n, f, k] * g[f, n, m] for f in range(F) for m in range(M)) / EPS
                assert den < EPS
                assert abs(H1[n, k, t] - H[n, k, t] * np.sqrt(num / EPS)) <= 1e-12 * H1[n, k, t]
    g1 = Dm.update_g(W1, H1, g, P)
    lam = fullcov.source_spectrogram(W1, H1)
    for f in range(F):
        for n in range(N):
            for m in range(M):
                num = sum(lam[f, t, n] * P[f, t, m] for t in range(T)) / EPS ** 2
                den = sum(lam[f, t, n] for t in range(T)) / EPS
                assert den < EPS
                assert abs(g1[f, n, m] - g[f, n, m] * np.sqrt(num / EPS)) <= 1e-12 * g1[f, n, m]


FLOOR_CHECKS = {
    "conventional_faint": lambda Dm: check_floored_stages_equal_conventional(Dm, faint_case),
    "conventional_loud": lambda Dm: check_floored_stages_equal_conventional(Dm, loud_case),
    "whitens": check_floored_model_whitens,
    "likelihood": check_floored_model_likelihood,
    "normaliser_single_mic": check_floored_normaliser_single_mic,
    "mm_closed_form": check_floored_mm_closed_form,
}


# ----------------------------------------------------------------- the cases really have their floors active
def test_faint_case_floors_model_and_every_denominator():
    mics = (3,)
    X, Q, g, W, H = faint_case(mics)
    assert np.all(_raw_model(W, H, g) < 1e-20)
    y = D.model_variance(D.source_psd(W, H), g)
    Q1 = D.ip_sweep(Q, D.weighted_covariances(X, y, mics), mics)
    P = D.powers(X, Q1, mics)
    for terms in (D.mm_terms_W, D.mm_terms_H, D.mm_terms_g):
        _, den = terms(W, H, g, P)
        assert np.all(den < 0.5 * EPS), terms.__name__


def test_loud_case_floors_every_normaliser():
    mics = (3,)
    X, Q, g, W, H = loud_case(mics)
    y = D.model_variance(D.source_psd(W, H), g)
    assert np.all(_raw_model(W, H, g) > 10 * EPS)
    V = D.weighted_covariances(X, y, mics)[0]
    Ql = D.q_blocks(Q, mics)[0]
    for mu in range(3):  # normaliser of each row as the sweep reaches it
        A = Ql @ V[:, mu]
        e = np.zeros((X.shape[0], 3))
        e[:, mu] = 1.0
        b = np.linalg.solve(A, e[..., None])[..., 0]
        s = np.einsum("fa,fab,fb->f", b.conj(), V[:, mu], b).real
        assert np.all(s < 0.1 * EPS), (mu, s)
        Ql = D.ip_update_row(Ql, V[:, mu], mu)


@pytest.mark.parametrize("name", sorted(FLOOR_CHECKS))
def test_floor_pin(name):
    FLOOR_CHECKS[name](D)
