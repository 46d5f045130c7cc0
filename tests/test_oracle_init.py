"""Pins of the oracle's initialisation (Sec. IV-A, steps 3, 5, 6) -- CPU only.

Each part is checked against what the mathematics fixes, not against its own formula:
* step 3: the time average of h = c^H R^-1 c / M is tr(R^-1 R) / M = 1 for every (f, n); h is
  unchanged when every c_ftn is multiplied by the same invertible matrix per bin (R changes
  with it); with one mic h = |c|^2 / mean_t |c|^2; R is the brute-force sum of outer products;
* step 5: the defining equations W^H B W = I and W^H A W = diag(lambda) with lambda ascending
  and the phase convention; one mic: w = 1 / sqrt(B), lambda = A / B; two mics: lambda are the
  roots of the quadratic det(A - lambda B) = 0, by the quadratic formula;
* step 6: with the problem posed as (R_N-1, R_N), ddiag(W^H R_N W) = 1 and ddiag(W^H R_N-1 W) =
  lambda exactly; every g entry equals the brute-force quadratic form w_mu^H R w_mu.
"""
import os
import types

import numpy as np
import pytest

from oracle import dfmnmf as D
from oracle import init as I
from paper_2605_19388_amd import synth


def _images(F=6, T=50, mics=(2, 3), N=3, K=2, seed=5, mixing="iid"):
    X, C = synth.source_images(F, T, mics, N, K, seed, mixing=mixing)
    return X, C


def check_image_covariances_brute_force(I):
    _, C = _images(F=2, T=7, mics=(2, 1), N=2)
    R = I.image_covariances(C)
    N, F, T, M = C.shape
    for f in range(F):
        for n in range(N):
            ref = sum(np.outer(C[n, f, t], C[n, f, t].conj()) for t in range(T)) / T
            np.testing.assert_allclose(R[f, n], ref, rtol=1e-13, atol=1e-15)


def check_spectrogram_time_average_is_one(I):
    _, C = _images()
    h = I.initial_spectrograms(C, I.image_covariances(C))
    np.testing.assert_allclose(h.mean(axis=2), 1.0, rtol=1e-9)  # solves with cond(R) up to ~1e6
    assert np.all(h > 0)


def check_spectrogram_invariant_to_a_linear_map_of_the_images(I):
    _, C = _images()
    rng = np.random.Generator(np.random.PCG64(3))
    N, F, T, M = C.shape
    A = rng.standard_normal((F, M, M)) + 1j * rng.standard_normal((F, M, M))
    C2 = np.einsum("fab,nftb->nfta", A, C)
    h1 = I.initial_spectrograms(C, I.image_covariances(C))
    h2 = I.initial_spectrograms(C2, I.image_covariances(C2))
    np.testing.assert_allclose(h2, h1, rtol=1e-9)


def check_spectrogram_single_mic(I):
    _, C = _images(mics=(1,), N=2)
    h = I.initial_spectrograms(C, I.image_covariances(C))
    p = np.abs(C[..., 0]) ** 2
    np.testing.assert_allclose(h, p / p.mean(axis=2, keepdims=True), rtol=1e-12)


def _hermitian_pd(rng, F, m):
    G = rng.standard_normal((F, m, 2 * m)) + 1j * rng.standard_normal((F, m, 2 * m))
    return np.einsum("fab,fcb->fac", G, G.conj()) / (2 * m)


def check_joint_diagonaliser_defining_equations(I, m):
    rng = np.random.Generator(np.random.PCG64(10 + m))
    A, B = _hermitian_pd(rng, 5, m), _hermitian_pd(rng, 5, m)
    for f in range(5):
        W, lam = I.joint_diagonaliser(A[f], B[f])
        np.testing.assert_allclose(W.conj().T @ B[f] @ W, np.eye(m), atol=1e-12)
        np.testing.assert_allclose(W.conj().T @ A[f] @ W, np.diag(lam), atol=1e-12)
        assert np.all(np.diff(lam) > 0)
        for mu in range(m):
            i = int(np.argmax(np.abs(W[:, mu])))
            assert abs(W[i, mu].imag) < 1e-14 and W[i, mu].real > 0


def check_joint_diagonaliser_one_mic(I):
    A, B = np.array([[3.0 + 0j]]), np.array([[4.0 + 0j]])
    W, lam = I.joint_diagonaliser(A, B)
    np.testing.assert_allclose(W, [[0.5]], rtol=1e-15)
    np.testing.assert_allclose(lam, [0.75], rtol=1e-15)


def check_joint_diagonaliser_two_mics_quadratic_formula(I):
    rng = np.random.Generator(np.random.PCG64(4))
    A, B = _hermitian_pd(rng, 1, 2)[0], _hermitian_pd(rng, 1, 2)[0]
    # det(A - l B) = det(B) l^2 - (a11 b22 + a22 b11 - a12 b21 - a21 b12) l + det(A)
    a2 = np.linalg.det(B).real
    a1 = -(A[0, 0] * B[1, 1] + A[1, 1] * B[0, 0] - A[0, 1] * B[1, 0] - A[1, 0] * B[0, 1]).real
    a0 = np.linalg.det(A).real
    disc = np.sqrt(a1 * a1 - 4 * a2 * a0)
    roots = np.sort([(-a1 - disc) / (2 * a2), (-a1 + disc) / (2 * a2)])
    _, lam = I.joint_diagonaliser(A, B)
    np.testing.assert_allclose(lam, roots, rtol=1e-12)


def check_initial_scm_of_the_last_two_sources(I, mics):
    """ddiag(W^H R_N W) = 1 and ddiag(W^H R_N-1 W) = lambda (ascending) in every block."""
    _, C = _images(F=4, T=80, mics=mics, N=3, mixing="delay")
    R = I.image_covariances(C)
    Q = I.initial_transform(R, mics)
    g = I.initial_scm(Q, R, mics)
    np.testing.assert_allclose(g[:, -1], 1.0, rtol=1e-10)
    for ml, (mo, _) in zip(mics, D.block_offsets(mics)):
        for f in range(4):
            sl = slice(mo, mo + ml)
            lam = np.linalg.eigvals(np.linalg.solve(R[f, -1, sl, sl], R[f, -2, sl, sl])).real
            np.testing.assert_allclose(g[f, -2, sl], np.sort(lam), rtol=1e-9)


def check_initial_scm_brute_force(I):
    mics = (2, 1)
    _, C = _images(F=3, T=40, mics=mics, N=3)
    R = I.image_covariances(C)
    Q = I.initial_transform(R, mics)
    g = I.initial_scm(Q, R, mics)
    for f in range(3):
        for n in range(3):
            for ml, (mo, qo) in zip(mics, D.block_offsets(mics)):
                for mu in range(ml):
                    q = Q[f, qo + mu * ml: qo + (mu + 1) * ml]   # row mu = w^H
                    w = q.conj()
                    val = sum(w[a].conj() * R[f, n, mo + a, mo + b] * w[b] for a in range(ml) for b in range(ml))
                    assert abs(g[f, n, mo + mu] - val.real) < 1e-12 * max(1.0, abs(val))


def check_initial_transform_needs_two_sources(I):
    _, C = _images(N=1)
    with pytest.raises(ValueError):
        I.initial_transform(I.image_covariances(C), (2, 3))


def check_initialised_model_reproduces_the_images_covariance_in_the_last_two_sources(I):
    """Q R_n Q^H is diagonal for the last two sources in every block: the model's SCMs
    Q^-1 diag(g_n) Q^-H reproduce their diagonal blocks exactly (eqs. (11)-(12))."""
    mics = (3, 2)
    _, C = _images(F=3, T=60, mics=mics, N=4)
    R = I.image_covariances(C)
    Q, g, _ = I.initialise(C, mics)
    for ml, (mo, qo) in zip(mics, D.block_offsets(mics)):
        sl = slice(mo, mo + ml)
        Ql = Q[:, qo:qo + ml * ml].reshape(3, ml, ml)
        Qi = np.linalg.inv(Ql)
        for n in (2, 3):
            model = np.einsum("fab,fb,fcb->fac", Qi, g[:, n, sl], Qi.conj())
            np.testing.assert_allclose(model, R[:, n, sl, sl], rtol=1e-9, atol=1e-12)


CHECKS = {
    "covariances": lambda Im: check_image_covariances_brute_force(Im),
    "time_average": lambda Im: check_spectrogram_time_average_is_one(Im),
    "linear_invariance": lambda Im: check_spectrogram_invariant_to_a_linear_map_of_the_images(Im),
    "single_mic": lambda Im: check_spectrogram_single_mic(Im),
    "gevd_m1": lambda Im: check_joint_diagonaliser_defining_equations(Im, 1),
    "gevd_m2": lambda Im: check_joint_diagonaliser_defining_equations(Im, 2),
    "gevd_m4": lambda Im: check_joint_diagonaliser_defining_equations(Im, 4),
    "gevd_one_mic": lambda Im: check_joint_diagonaliser_one_mic(Im),
    "gevd_quadratic": lambda Im: check_joint_diagonaliser_two_mics_quadratic_formula(Im),
    "scm_last_two_2x3": lambda Im: check_initial_scm_of_the_last_two_sources(Im, (2, 3)),
    "scm_last_two_4x4": lambda Im: check_initial_scm_of_the_last_two_sources(Im, (4, 4, 4, 4)),
    "scm_last_two_112": lambda Im: check_initial_scm_of_the_last_two_sources(Im, (1, 1, 2)),
    "scm_brute_force": lambda Im: check_initial_scm_brute_force(Im),
    "two_sources": lambda Im: check_initial_transform_needs_two_sources(Im),
    "model_reproduces": lambda Im: check_initialised_model_reproduces_the_images_covariance_in_the_last_two_sources(Im),
}


@pytest.mark.parametrize("name", sorted(CHECKS))
def test_pin(name):
    CHECKS[name](I)


# Plausible mistakes planted in a copy of oracle/init.py (built in memory); each must fail a pin.
SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "init.py")
MUTANTS = {
    "covariance_conj_on_wrong_side": ('"nfta,nftb->fnab", C, C.conj()', '"nfta,nftb->fnab", C.conj(), C'),
    "covariance_1_over_T_dropped": ("optimize=True) / T", "optimize=True)"),
    "spectrogram_1_over_M_dropped": (".real / M", ".real"),
    "spectrogram_without_inverse": ("u = np.linalg.solve(R[f, n], C[n, f].T)", "u = C[n, f].T"),
    "gevd_pencil_swapped": ("joint_diagonaliser(R[f, N - 2, sl, sl], R[f, N - 1, sl, sl])",
                            "joint_diagonaliser(R[f, N - 1, sl, sl], R[f, N - 2, sl, sl])"),
    "gevd_descending": ("lam, W = scipy.linalg.eigh(A, B)", "lam, W = scipy.linalg.eigh(A, B)\n    lam, W = lam[::-1], W[:, ::-1]"),
    "gevd_phase_not_fixed": ("W[:, mu] = _fix_phase(W[:, mu])", "W[:, mu] = W[:, mu] * 1j"),
    "Q_not_conjugate_transposed": ("Q[f, qo:qo + ml * ml] = W.conj().T.reshape(-1)", "Q[f, qo:qo + ml * ml] = W.T.reshape(-1)"),
    "scm_conjugates_swapped": ('"fua,fnab,fub->fnu", Ql, R[:, :, sl, sl], Ql.conj()', '"fua,fnab,fub->fnu", Ql.conj(), R[:, :, sl, sl], Ql'),
    "scm_wrong_source": ("Ql, R[:, :, sl, sl], Ql.conj()", "Ql, R[:, ::-1, sl, sl], Ql.conj()"),
}


def _mutant(old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("oracle.init_mutant")
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(old, new), "init_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(name):
    mod = _mutant(*MUTANTS[name])
    failed = []
    for check, fn in CHECKS.items():
        try:
            fn(mod)
        except (AssertionError, ValueError, np.linalg.LinAlgError):
            failed.append(check)
    assert failed, f"mutant {name} passes every pin"
