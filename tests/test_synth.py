"""Seeded input generator: determinism, shapes and the statistics of the recipe (CPU only)."""
import numpy as np
import pytest

from paper_2605_19388_amd import synth


def test_deterministic_and_seed_sensitive():
    a = synth.mixture(5, 30, (2, 2), 2, 3, seed=4)
    b = synth.mixture(5, 30, (2, 2), 2, 3, seed=4)
    c = synth.mixture(5, 30, (2, 2), 2, 3, seed=5)
    assert np.array_equal(a, b)
    assert not np.allclose(a, c)


def test_workload_shapes():
    for name, wl in synth.WORKLOADS.items():
        p = synth.make(name, T=20, F=7)
        assert p["X"].shape == (7, 20, wl.M) and p["X"].dtype == np.complex128
        assert p["Q"].shape == (7, sum(m * m for m in wl.mics))
        assert p["g"].shape == (7, wl.N, wl.M) and np.all(p["g"] == 1.0)
        assert p["W"].shape == (wl.N, 7, wl.K) and np.all(p["W"] > 0)
        assert p["H"].shape == (wl.N, wl.K, 20) and np.all(p["H"] > 0)


def test_initial_q_is_block_identity():
    Q, _, _, _ = synth.initial_state(3, 4, (2, 3), 2, 2, seed=0)
    off = synth.qblock_offsets((2, 3))
    assert off == [0, 4]
    np.testing.assert_array_equal(Q[:, 0:4].reshape(3, 2, 2), np.broadcast_to(np.eye(2), (3, 2, 2)))
    np.testing.assert_array_equal(Q[:, 4:13].reshape(3, 3, 3), np.broadcast_to(np.eye(3), (3, 3, 3)))


def test_noise_only_statistics():
    """With no sources the mixture is CN(0, 1e-3 I): mean power 1e-3, circular."""
    X = synth.mixture(64, 400, (2, 2), 0, 1, seed=9)
    p = np.mean(np.abs(X) ** 2)
    assert abs(p / 1e-3 - 1) < 0.02
    assert abs(np.mean(X.real ** 2) - np.mean(X.imag ** 2)) < 0.03 * 1e-3


def test_delay_mixing_is_unit_modulus_times_gain():
    """Steering vectors: |a| equals the per-(subarray, source) gain in [0.5, 2]; DC bin has no phase."""
    F, T, mics, N = 9, 4, (2, 2), 3
    rng = np.random.Generator(np.random.PCG64(3))
    rng.gamma(1.0, 1.0, size=(N, F, 1))
    rng.gamma(1.0, 1.0, size=(N, 1, T))
    X = synth.mixture(F, T, mics, N, 1, seed=3, mixing="delay", noise=0.0)
    # at f = 0 all mics of one subarray see the same gain-weighted sum: ratio between mics is real
    r = X[0, :, 1] / X[0, :, 0]
    assert np.allclose(r.imag, 0.0, atol=1e-9)


@pytest.mark.parametrize("dist, conv, m", [("paper_4x4", "paper_16", 16), ("table2", "table2_12", 12)])
def test_conventional_workload_shares_the_recording(dist, conv, m):
    """paper_16 and table2_12 separate the very recordings of paper_4x4 and table2 with one block
    of all the mics (L = 1)."""
    a = synth.make(dist, T=40, F=33)
    b = synth.make(conv, T=40, F=33)
    assert np.array_equal(a["X"], b["X"])
    assert b["mics"] == (m,) and b["Q"].shape == (33, m * m)
    assert np.array_equal(b["Q"][:, ::m + 1], np.ones((33, m)))  # identity block
    assert np.array_equal(a["W"], b["W"]) and np.array_equal(a["H"], b["H"])
