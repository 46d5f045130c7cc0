"""Tile autotuner for distributed FastMNMF plans.

The one tile parameter of a plan is ``tile``, the largest number of frames per slice of the
streaming kernels (16, 32, 64 or 128; the library keeps the largest that fits its LDS budget at
or below it).  It sets how many workgroups the per-frame kernels launch and how long each one's
frame loop is, so the best value depends on the recording length T and on (N, M).  ``tune``
measures each candidate on a synthetic mixture of the shape (seeded, from ``synth``) by timing
``dfm_step`` with HIP events and returns the fastest; results are cached per shape class (bins
of T, the partition, N, K, precision and flags), in memory and optionally in a JSON file.
"""
from __future__ import annotations

import json
import os

CANDIDATES = (16, 32, 64, 128)
T_BIN = 250  # recordings within one bin of T share a tuned tile

_cache: dict = {}


def shape_key(F, T, mics, N, K, fp32=True, flags=0):
    return (int(F), int(T) // T_BIN, tuple(int(m) for m in mics), int(N), int(K), bool(fp32), int(flags))


def choose(timings: dict) -> int:
    """The fastest candidate (the larger tile on a tie)."""
    return min(timings, key=lambda c: (timings[c], -c))


def _measure(X, Q, g, W, H, mics, N, K, flags, tile, iters, reps):
    import torch

    from .binding import DistributedFastMNMF
    p = DistributedFastMNMF(X, mics, N, K, W=W, H=H, Q=Q, g=g, flags=flags, tile=tile)
    p.step(1)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        p.step(iters)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / iters)
    p.close()
    return best


def tune(F, T, mics, N, K, fp32=True, flags=0, candidates=CANDIDATES, iters=3, reps=2, seed=0, cache_path=None):
    """Best tile for the shape class of (F, T, mics, N, K, precision, flags), and the per-candidate
    milliseconds per iteration it was chosen from (empty if it came from the cache)."""
    key = shape_key(F, T, mics, N, K, fp32, flags)
    skey = repr(key)
    if skey in _cache:
        return _cache[skey], {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            stored = json.load(fh)
        if skey in stored:
            _cache[skey] = int(stored[skey])
            return _cache[skey], {}
    import numpy as np

    from . import synth
    X = synth.mixture(F, T, mics, N, K, seed, mixing="delay")
    Q, g, W, H = synth.initial_state(F, T, mics, N, K, seed + 1)
    cdt, rdt = (np.complex64, np.float32) if fp32 else (np.complex128, np.float64)
    X, Q, g, W, H = X.astype(cdt), Q.astype(cdt), g.astype(rdt), W.astype(rdt), H.astype(rdt)
    timings = {c: _measure(X, Q, g, W, H, mics, N, K, flags, c, iters, reps) for c in candidates}
    best = choose(timings)
    _cache[skey] = best
    if cache_path:
        stored = {}
        if os.path.exists(cache_path):
            with open(cache_path) as fh:
                stored = json.load(fh)
        stored[skey] = best
        with open(cache_path, "w") as fh:
            json.dump(stored, fh, indent=1)
    return best, timings
