"""Seeded synthetic mixtures and initial parameters for distributed FastMNMF.

This module only draws random numbers and mixes them into observations the way
the local Gaussian generative model of Sec. II-A (eqs. (1)-(2)) describes a
multichannel recording: sources with NMF power spectrograms, each reaching the
microphones through a mixing vector, plus a little white sensor noise.  It holds
none of the estimation method's arithmetic, so both the FP64 oracle and the HIP
path can take their inputs from it.

All draws use ``numpy.random.Generator(PCG64(seed))``, which is bit-reproducible
across machines.

Workloads (names are what they are, sizes in the name):

* ``small_2x2`` -- F=129, T=200, two subarrays of two mics (M=4), N=2, K=4.
  Mixing vectors i.i.d. CN(0, 1) per entry.
* ``paper_4x4`` -- F=513 (1024-point STFT), T=625, four subarrays of four mics
  (M=16), N=5, K=16.  Mixing vectors are steering vectors with a random delay
  in [0, 20] samples per (source, mic) and a gain in [0.5, 2] per
  (subarray, source); with five sources every 4-mic subarray is locally
  underdetermined, as in the paper's five-source condition (Sec. IV-A).
* ``paper_16`` -- the same recording (drawn exactly as ``paper_4x4``) with one
  16-mic block: the conventional, non-distributed method (L = 1).
* ``table2`` -- the shape of the paper's runtime comparison (Sec. IV, Table II):
  F=2049 (4096-point STFT), T=157, three subarrays of four mics (M=12), N=3,
  K=16, 200 iterations; mixing as ``paper_4x4``.
* ``table2_12`` -- the same recording with one 12-mic block: the method that
  Table II compares against (all subarrays' mics as one array).

Sources: s_ftn ~ CN(0, (W*_n H*_n)_ft) with W*_n ~ Gamma(1,1)[F,K] and
H*_n ~ Gamma(1,1)[K,T]; x_ft = sum_n a_fn s_ftn + CN(0, 1e-3 I).
Initial parameters: Q_f = I (block-diagonal identity), g = 1, and W0, H0 drawn
Gamma(1, 1) from a second generator seeded with ``seed + 1``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["Workload", "WORKLOADS", "mixture", "source_images", "initial_state", "make", "qblock_offsets"]


@dataclass(frozen=True)
class Workload:
    name: str
    F: int
    T: int
    mics: tuple
    N: int
    K: int
    mixing: str          # "iid" or "delay"
    seed: int
    iters: int
    noise: float = 1e-3
    extra: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(sum(self.mics))

    @property
    def bins(self) -> int:
        """F*T*M: the number of time-frequency-microphone bins."""
        return self.F * self.T * self.M


WORKLOADS = {
    "small_2x2": Workload("small_2x2", F=129, T=200, mics=(2, 2), N=2, K=4,
                          mixing="iid", seed=0, iters=10),
    "paper_4x4": Workload("paper_4x4", F=513, T=625, mics=(4, 4, 4, 4), N=5, K=16,
                          mixing="delay", seed=1, iters=100),
    # The same recording as paper_4x4 (drawn with its four-subarray steering), separated
    # with one 16-mic block: the conventional FastMNMF the paper compares against.
    "paper_16": Workload("paper_16", F=513, T=625, mics=(16,), N=5, K=16,
                         mixing="delay", seed=1, iters=100, extra={"data_mics": (4, 4, 4, 4)}),
    "table2": Workload("table2", F=2049, T=157, mics=(4, 4, 4), N=3, K=16,
                       mixing="delay", seed=5, iters=200),
    "table2_12": Workload("table2_12", F=2049, T=157, mics=(12,), N=3, K=16,
                          mixing="delay", seed=5, iters=200, extra={"data_mics": (4, 4, 4)}),
}


def _cn(rng: np.random.Generator, shape, var=1.0) -> np.ndarray:
    """Circular complex normal CN(0, var): real and imaginary parts N(0, var/2)."""
    s = np.sqrt(np.asarray(var, dtype=np.float64) / 2.0)
    return s * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def qblock_offsets(mics) -> list:
    """Offset of each subarray's M_l x M_l block inside one frequency's packed Q row."""
    offs, o = [], 0
    for ml in mics:
        offs.append(o)
        o += ml * ml
    return offs


def mixture(F: int, T: int, mics, N: int, K: int, seed: int, mixing: str = "iid",
            noise: float = 1e-3, max_delay: float = 20.0, gain_range=(0.5, 2.0), _masks: bool = False):
    """Return X[F, T, M] complex128 drawn from the generative model of eqs. (1)-(2).

    With ``_masks`` also return the sources' share of the power at each (f, t),
    psd_n / sum_n' psd_n' [N, F, T], from the same draws (see ``source_images``)."""
    mics = tuple(int(m) for m in mics)
    M = sum(mics)
    rng = np.random.Generator(np.random.PCG64(seed))
    Wt = rng.gamma(1.0, 1.0, size=(N, F, K))
    Ht = rng.gamma(1.0, 1.0, size=(N, K, T))
    psd = np.zeros((F, T, N))
    for n in range(N):
        psd[:, :, n] = Wt[n] @ Ht[n]                                       # [F, T, N]
    s = _cn(rng, (F, T, N), psd)
    if mixing == "iid":
        A = _cn(rng, (F, N, M))
    elif mixing == "delay":
        nfft = 2 * (F - 1) if F > 1 else 2
        tau = rng.uniform(0.0, max_delay, size=(N, M))                   # per (source, mic)
        gain = rng.uniform(gain_range[0], gain_range[1], size=(len(mics), N))
        gmic = np.repeat(gain, mics, axis=0).T                           # [N, M]
        f = np.arange(F, dtype=np.float64)[:, None, None]
        A = gmic[None] * np.exp(-2j * np.pi * f * tau[None] / nfft)      # [F, N, M]
    else:
        raise ValueError(f"unknown mixing {mixing!r}")
    X = np.einsum("fnm,ftn->ftm", A, s) + _cn(rng, (F, T, M), noise)
    if _masks:
        return np.ascontiguousarray(X), np.transpose(psd / psd.sum(axis=2, keepdims=True), (2, 0, 1))
    return np.ascontiguousarray(X)


def source_images(F: int, T: int, mics, N: int, K: int, seed: int, mixing: str = "iid", **kw):
    """Estimates of the N source images c_ftn [N, F, T, M] complex128 of the recording that
    ``mixture`` draws with the same arguments, made the way the paper's initialisation makes
    them (Sec. IV-A, step 2: soft time-frequency masks applied to the mixture): c_ftn = m_ftn x_ft
    with the mask m_ftn = psd_ftn / sum_n psd_ftn taken from the sources' true power
    spectrograms.  (The paper estimates the masks by clustering; that step is a separate
    method and stands outside this library.)  Returns (X, C)."""
    X, m = mixture(F, T, mics, N, K, seed, mixing=mixing, _masks=True, **kw)
    return X, np.ascontiguousarray(m[:, :, :, None] * X[None])


def initial_state(F: int, T: int, mics, N: int, K: int, seed: int):
    """Q = block identity [F, sum M_l^2] complex, g = 1 [F, N, M], W0 [N, F, K], H0 [N, K, T]."""
    mics = tuple(int(m) for m in mics)
    M = sum(mics)
    Q = np.zeros((F, sum(m * m for m in mics)), dtype=np.complex128)
    for ml, off in zip(mics, qblock_offsets(mics)):
        for mu in range(ml):
            Q[:, off + mu * ml + mu] = 1.0
    g = np.ones((F, N, M), dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    W = rng.gamma(1.0, 1.0, size=(N, F, K))
    H = rng.gamma(1.0, 1.0, size=(N, K, T))
    return Q, g, W, H


def make(workload, seed: int | None = None, T: int | None = None, F: int | None = None):
    """Mixture and initial state for a named workload (or a Workload), optionally resized.

    Returns a dict with X, Q, g, W, H (float64 / complex128) and the shape fields.
    """
    wl = WORKLOADS[workload] if isinstance(workload, str) else workload
    seed = wl.seed if seed is None else seed
    F = wl.F if F is None else F
    T = wl.T if T is None else T
    X = mixture(F, T, wl.extra.get("data_mics", wl.mics), wl.N, wl.K, seed, mixing=wl.mixing, noise=wl.noise)
    Q, g, W, H = initial_state(F, T, wl.mics, wl.N, wl.K, seed + 1)
    return dict(X=X, Q=Q, g=g, W=W, H=H, mics=tuple(wl.mics), N=wl.N, K=wl.K,
                F=F, T=T, M=wl.M, name=wl.name, iters=wl.iters)
