"""Helpers for the GPU tests: build plans through the C ABI and compare with the oracle."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

from oracle import dfmnmf as D


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"


def announce(what: str):
    print(f"\n[gpu] {what}", file=sys.stderr, flush=True)


def as_precision(a, fp32: bool):
    """Round an input to the precision the GPU path stores it in, then back to FP64 for the oracle."""
    a = np.asarray(a)
    if not fp32:
        return a.astype(np.complex128 if np.iscomplexobj(a) else np.float64)
    if np.iscomplexobj(a):
        return a.astype(np.complex64).astype(np.complex128)
    return a.astype(np.float32).astype(np.float64)


def plan(X, mics, N, K, Q, g, W, H, fp32: bool, eps=1e-6, flags=0):
    from paper_2605_19388_amd import DistributedFastMNMF
    cdt = np.complex64 if fp32 else np.complex128
    rdt = np.float32 if fp32 else np.float64
    return DistributedFastMNMF(np.asarray(X, dtype=cdt), mics, N, K,
                               W=np.asarray(W, dtype=rdt), H=np.asarray(H, dtype=rdt),
                               Q=np.asarray(Q, dtype=cdt), g=np.asarray(g, dtype=rdt), eps=eps, flags=flags)


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def max_rel(a, b, floor=0.0):
    """Largest elementwise |a-b| / max(|b|, floor)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor)))


def elem_rel(a, b):
    """Largest elementwise |a-b| / |b| of a positive reference (W, H, g)."""
    b = np.asarray(b)
    assert np.all(b > 0)
    return float(np.max(np.abs(np.asarray(a) - b) / b))


def q_block_errors(got, ref, mics):
    """err[f, l] = max |got - ref| / max |ref| over the entries of block (f, l) of Q [F][sum M_l^2]."""
    err = np.zeros((got.shape[0], len(mics)))
    off = 0
    for l, ml in enumerate(mics):
        g, r = got[:, off:off + ml * ml], ref[:, off:off + ml * ml]
        err[:, l] = np.abs(g - r).max(axis=1) / np.abs(r).max(axis=1)
        off += ml * ml
    return err


def per_bin_errors(got, ref, axes):
    """max over `axes` of |got - ref| divided by max over `axes` of |ref| (one value per remaining index)."""
    return np.abs(got - ref).max(axis=axes) / np.abs(ref).max(axis=axes)


REPORT_FILE = os.environ.get("DFM_PARITY_REPORT")


def report(line: str):
    """Worst-bin errors and condition numbers of a parity case: to stderr, and appended to the file
    named by DFM_PARITY_REPORT if set."""
    print(f"[parity] {line}", file=sys.stderr, flush=True)
    if REPORT_FILE:
        with open(REPORT_FILE, "a") as fh:
            fh.write(line + "\n")


def nll_rel(got, ref, F, T, M):
    return abs(got - ref) / max(abs(ref), F * T * M)


def oracle_stage(stage, X, mics, state, eps=1e-6):
    """Apply one stage of the oracle to `state` (dict of Q, g, W, H in FP64); returns the new state."""
    Q, g, W, H = state["Q"], state["g"], state["W"], state["H"]
    if stage == "ip":
        y = D.model_variance(D.source_psd(W, H), g, eps)
        Q = D.ip_sweep(Q, D.weighted_covariances(X, y, mics), mics, eps)
    elif stage == "W":
        W = D.update_W(W, H, g, D.powers(X, Q, mics), eps)
    elif stage == "H":
        H = D.update_H(W, H, g, D.powers(X, Q, mics), eps)
    elif stage == "g":
        g = D.update_g(W, H, g, D.powers(X, Q, mics), eps)
    else:
        raise ValueError(stage)
    return dict(Q=Q, g=g, W=W, H=H)


def state64(p):
    """GPU state as FP64 numpy arrays."""
    s = p.state()
    return {k: v.astype(np.complex128 if np.iscomplexobj(v) else np.float64) for k, v in s.items()}


STAGE_KEY = {"ip": "Q", "W": "W", "H": "H", "g": "g"}

gpu = pytest.mark.gpu
