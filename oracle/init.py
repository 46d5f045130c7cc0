"""Initial parameters of distributed FastMNMF from estimates of the source images -- TEST
INFRASTRUCTURE (only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import it; the library never does).

Sec. IV-A describes the initialisation in six steps.  Steps 1-2 (masks by clustering, soft
masking) and 4 (Itakura-Saito NMF of the initial spectrograms) are separate methods outside this
library; steps 3, 5 and 6 turn source-image estimates c_ftn (C [N, F, T, M]) into the initial
spectrograms, transformations and diagonalised SCMs:

* step 3 -- R_fn = (1/T) sum_t c_ftn c_ftn^H (full M x M, also across subarrays) and
  h_ftn = c_ftn^H R_fn^{-1} c_ftn / M;
* step 5 -- for every bin f and subarray l, the matrix W_fl whose columns jointly diagonalise the
  l-th diagonal blocks of R_f,N-1 and R_f,N (the last two sources) by the generalized eigenvalue
  problem R_f,N-1^(l) w = lambda R_f,N^(l) w; Q_fl = W_fl^H (row mu is w_mu^H);
* step 6 -- Lambda_fn^(l) = ddiag(W_fl^H R_fn^(l) W_fl), i.e. g[f, n, o_l + mu] = w_mu^H R_fn^(l) w_mu.

Readings where the paper is silent (listed with the design notes): the problem is taken as
A w = lambda B w with A = R_f,N-1^(l), B = R_f,N^(l), eigenvectors normalised to W^H B W = I,
eigenvalues in ascending order (the rows of Q_fl in that order), and each eigenvector's phase
fixed so that its entry of largest modulus (the first such entry on a tie) is real and positive.
The cost (13) and the separated images do not depend on these choices (a row's phase or the
order of the rows rescale or permute the model's diagonal), but Q itself does.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .dfmnmf import block_offsets


def image_covariances(C):
    """R[f, n] = (1/T) sum_t c_ftn c_ftn^H for C [N, F, T, M] (step 3).  Returns [F, N, M, M]."""
    T = C.shape[2]
    return np.einsum("nfta,nftb->fnab", C, C.conj(), optimize=True) / T


def initial_spectrograms(C, R):
    """h[n, f, t] = c_ftn^H R_fn^{-1} c_ftn / M (step 3).  Returns [N, F, T] real."""
    N, F, T, M = C.shape
    h = np.empty((N, F, T))
    for n in range(N):
        for f in range(F):
            u = np.linalg.solve(R[f, n], C[n, f].T)             # [M, T]: R^{-1} c_t
            h[n, f] = np.einsum("tm,mt->t", C[n, f].conj(), u).real / M
    return h


def _fix_phase(w):
    """Scale eigenvector w by a unit complex number so that its entry of largest modulus (the first
    such entry) is real and positive."""
    i = int(np.argmax(np.abs(w)))
    return w * (np.conj(w[i]) / abs(w[i]))


def joint_diagonaliser(A, B):
    """Columns w_mu of W [m, m] solve A w = lambda B w (A Hermitian, B Hermitian positive definite),
    with W^H B W = I, lambda ascending and each column's phase fixed (_fix_phase).  Returns
    (W, lambda)."""
    lam, W = scipy.linalg.eigh(A, B)
    for mu in range(W.shape[1]):
        W[:, mu] = _fix_phase(W[:, mu])
    return W, lam


def initial_transform(R, mics):
    """Q [F, sum_l M_l^2]: block l of bin f is W_fl^H from the l-th diagonal blocks of R[f, N-2]
    and R[f, N-1] (step 5; the paper's sources N-1 and N, counted from one)."""
    F, N = R.shape[:2]
    if N < 2:
        raise ValueError("the joint diagonalisation of step 5 needs at least two sources")
    Q = np.zeros((F, sum(m * m for m in mics)), dtype=np.complex128)
    for ml, (mo, qo) in zip(mics, block_offsets(mics)):
        sl = slice(mo, mo + ml)
        for f in range(F):
            W, _ = joint_diagonaliser(R[f, N - 2, sl, sl], R[f, N - 1, sl, sl])
            Q[f, qo:qo + ml * ml] = W.conj().T.reshape(-1)
    return Q


def initial_scm(Q, R, mics):
    """g[f, n, o_l + mu] = w_mu^H R_fn^(l) w_mu (step 6: ddiag of W_fl^H R_fn^(l) W_fl), real."""
    F, N, M, _ = R.shape
    g = np.zeros((F, N, M))
    for ml, (mo, qo) in zip(mics, block_offsets(mics)):
        sl = slice(mo, mo + ml)
        Ql = Q[:, qo:qo + ml * ml].reshape(F, ml, ml)            # rows w_mu^H
        g[:, :, sl] = np.einsum("fua,fnab,fub->fnu", Ql, R[:, :, sl, sl], Ql.conj(), optimize=True).real
    return g


def initialise(C, mics):
    """Steps 3, 5 and 6 for source-image estimates C [N, F, T, M]: returns (Q, g, h)."""
    R = image_covariances(C)
    Q = initial_transform(R, mics)
    return Q, initial_scm(Q, R, mics), initial_spectrograms(C, R)
