"""Shared test helpers: tiny random problems and layout conversions (test code only)."""
from __future__ import annotations

import numpy as np

from paper_2605_19388_amd import synth


def random_state(F, T, mics, N, K, seed, q_scale=0.3):
    """A generic (non-identity) state: block Q = I + noise, random positive g, W, H."""
    rng = np.random.Generator(np.random.PCG64(seed))
    offs = synth.qblock_offsets(mics)
    Q = np.zeros((F, sum(m * m for m in mics)), dtype=np.complex128)
    for ml, off in zip(mics, offs):
        B = np.eye(ml)[None] + q_scale * (rng.standard_normal((F, ml, ml))
                                          + 1j * rng.standard_normal((F, ml, ml)))
        Q[:, off:off + ml * ml] = B.reshape(F, -1)
    M = sum(mics)
    g = rng.uniform(0.5, 2.0, size=(F, N, M))
    W = rng.gamma(1.0, 1.0, size=(N, F, K)) + 0.1
    H = rng.gamma(1.0, 1.0, size=(N, K, T)) + 0.1
    return Q, g, W, H


def tiny_problem(F=3, T=40, mics=(2, 3), N=2, K=3, seed=7, mixing="iid"):
    X = synth.mixture(F, T, mics, N, K, seed, mixing=mixing)
    Q, g, W, H = random_state(F, T, mics, N, K, seed + 100)
    return X, Q, g, W, H


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))
