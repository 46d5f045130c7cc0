"""Brute-force checks from the full spatial covariance matrices.

TEST INFRASTRUCTURE.  Builds R_in and the observation covariance of eq. (1)
explicitly, M x M per time-frequency point, so that the diagonalised cost
(13), the powers |Q x|^2 and the Wiener filter can be pinned to the
generative model itself.  Tiny inputs only.
"""
from __future__ import annotations

import numpy as np


def blockdiag_transform(blocks):
    """W_i^H = blkdiag(Q_f1, ..., Q_fL) for every f: [F, M, M] (Sec. III-B)."""
    F = blocks[0].shape[0]
    M = sum(b.shape[1] for b in blocks)
    out = np.zeros((F, M, M), dtype=np.complex128)
    o = 0
    for b in blocks:
        ml = b.shape[1]
        out[:, o:o + ml, o:o + ml] = b
        o += ml
    return out


def spatial_covariances(Qfull, g):
    """R_fn = Q_f^{-1} diag(g_fn) Q_f^{-H}, the joint-diagonalisation form of eq. (3)."""
    F, N, M = g.shape
    R = np.empty((F, N, M, M), dtype=np.complex128)
    for f in range(F):
        Qi = np.linalg.inv(Qfull[f])
        for n in range(N):
            R[f, n] = Qi @ np.diag(g[f, n]) @ Qi.conj().T
    return R


def source_spectrogram(W, H):
    """h_ftn = sum_k W[n,f,k] H[n,k,t], eq. (2), as an explicit loop over k."""
    N, F, K = W.shape
    T = H.shape[2]
    h = np.zeros((F, T, N))
    for n in range(N):
        for k in range(K):
            h[:, :, n] += np.outer(W[n, :, k], H[n, k, :])
    return h


def nll_fullcov(X, Qfull, g, W, H):
    """sum_{f,t} [x^H S^{-1} x + ln det S] with S = sum_n h_ftn R_fn (eq. (1) without the M ln pi constant)."""
    F, T, M = X.shape
    R = spatial_covariances(Qfull, g)
    h = source_spectrogram(W, H)
    total = 0.0
    for f in range(F):
        for t in range(T):
            S = np.einsum("n,nab->ab", h[f, t], R[f])
            x = X[f, t]
            total += float(np.real(x.conj() @ np.linalg.solve(S, x)))
            total += float(np.linalg.slogdet(S)[1])
    return total


def wiener_fullcov(X, Qfull, g, W, H):
    """Posterior means E[c_ftn | x_ft] = h R_fn S^{-1} x under eq. (1): [N, F, T, M]."""
    F, T, M = X.shape
    N = W.shape[0]
    R = spatial_covariances(Qfull, g)
    h = source_spectrogram(W, H)
    C = np.empty((N, F, T, M), dtype=np.complex128)
    for f in range(F):
        for t in range(T):
            S = np.einsum("n,nab->ab", h[f, t], R[f])
            u = np.linalg.solve(S, X[f, t])
            for n in range(N):
                C[n, f, t] = h[f, t, n] * (R[f, n] @ u)
    return C


def jointly_diagonalizable(Rs, tol=1e-9):
    """Commutator test of the appendix theorem.

    With S = sum_n R_n positive definite, R_1..R_N are jointly diagonalisable
    iff the whitened S^{-1/2} R_n S^{-1/2} pairwise commute.
    """
    S = sum(Rs)
    wv, U = np.linalg.eigh(S)
    Sih = U @ np.diag(wv ** -0.5) @ U.conj().T
    Rt = [Sih @ R @ Sih for R in Rs]
    scale = max(np.linalg.norm(R) for R in Rt)
    for a in range(len(Rt)):
        for b in range(a + 1, len(Rt)):
            if np.linalg.norm(Rt[a] @ Rt[b] - Rt[b] @ Rt[a]) > tol * scale * scale:
                return False
    return True
