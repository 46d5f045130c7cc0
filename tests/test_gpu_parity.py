"""HIP path vs the FP64 oracle through the C ABI (GPU only).

One-step parity restarts the oracle from the GPU's own state before every stage,
so each kernel's error is measured alone; end-to-end parity runs both sides from
the same seeded inputs.  Tolerances:

* FP64 path: 1e-10 relative (rounding order only); Q, the output of a backward-stable
  solve, is held to max(1e-10, 1e-15 * M_l * kappa) with kappa defined below.
* FP32 path, one stage: sums of positive terms in FP32 carry ~u*sqrt(n) relative
  error (u = 6e-8, n <= a few thousand terms) -> 2e-5 for W, H, g.  The FP32
  covariances (relative error ~u*sqrt(SL) <= ~1e-6 per slice of SL <= 128
  frames) feed an FP64 solve that amplifies it by kappa = max(cond(Q V_mu),
  cond(V_mu)), so Q is
  held to max(2e-4, 2e-8 * kappa) with kappa measured by the oracle on the same
  inputs; the cost after the sweep, which is flat to first order along the
  ill-determined directions, is held to max(1e-6, 1e-9 * kappa) relative.
* FP32 end to end: 1e-4 relative on the cost and on each source's separated
  spectrogram, the bar the method is held to.
"""
import os

import numpy as np
import pytest
import torch

from oracle import dfmnmf as D
from paper_2605_19388_amd import synth
from tests.common import random_state
from tests.gpu_common import (STAGE_KEY, announce, as_precision, nll_rel, oracle_stage, plan, rel,
                              require_gpu, state64)

pytestmark = pytest.mark.gpu

TOL_STAGE = {False: {"Q": 1e-10, "W": 1e-11, "H": 1e-11, "g": 1e-11},
             True: {"Q": 2e-4, "W": 2e-5, "H": 2e-5, "g": 2e-5}}


@pytest.fixture(autouse=True)
def _gpu(request):
    require_gpu()
    announce(request.node.nodeid)
    yield
    torch.cuda.synchronize()


def _problem(F, T, mics, N, K, seed, fp32, mixing="iid"):
    X = synth.mixture(F, T, mics, N, K, seed, mixing=mixing)
    Q, g, W, H = random_state(F, T, mics, N, K, seed + 1)
    X, Q, g, W, H = (as_precision(a, fp32) for a in (X, Q, g, W, H))
    return X, Q, g, W, H


def _ip_condition(X, mics, st):
    """max over (f, l, mu) of cond(Q_fl V_flmu) and cond(V_flmu): the amplification of
    covariance errors in the solve of eq. (15), (Q V) b = e  <=>  V b = Q^{-1} e."""
    y = D.model_variance(D.source_psd(st["W"], st["H"]), st["g"])
    V = D.weighted_covariances(X, y, mics)
    Qb = D.q_blocks(st["Q"], mics)
    return max(max(float(np.linalg.cond(Qb[l] @ V[l][:, mu]).max()), float(np.linalg.cond(V[l][:, mu]).max()))
               for l in range(len(mics)) for mu in range(mics[l]))


# ------------------------------------------------------------------ one-step parity per stage
STAGE_CASES = [
    # (F, T, mics, N, K): several slices with a ragged tail, F not a multiple of the
    # 16-bin activation tiles.  Generic kernels: mixed or unlisted shapes.
    (37, 301, (2, 3, 1), 3, 4),
    (5, 260, (16,), 2, 3),
    (3, 40, (1, 1, 1, 1), 2, 2),
    # Shape-specialised kernels, one case per compiled (N, K, M_l) set.
    (9, 97, (4, 4, 4, 4), 5, 16),
    (37, 301, (4, 4, 4, 4), 5, 16),
    (18, 150, (16,), 5, 16),
    (20, 77, (4, 4), 3, 16),
    (20, 77, (4, 4, 4), 8, 16),
    (21, 50, (4, 4, 4), 3, 16),
    # W[n] over more than one LDS window in the H update (FP64 above 176 bins, FP32 above 592):
    # the bin-split H update.
    (200, 37, (4, 4, 4), 3, 16),
    (620, 21, (4, 4, 4), 3, 16),
    # H[n] over more than one LDS window in the W update (k_wgemm_f walks the windows; FP64 above
    # 224 frames, FP32 above 736).
    (5, 800, (4, 4, 4, 4), 5, 16),
    (33, 130, (2, 2), 2, 4),
    # Fewer frames per bin than a g-update workgroup's range: ranges span up to six bins.
    (23, 9, (4, 4, 4, 4), 5, 16),
    (7, 3, (2, 2), 2, 4),
]

FAST = ["k_gramd_f", "k_ip_f", "k_pw_f", "k_wgemm_f", "k_h_f", "k_hgemm_f", "k_g_f"]
GENERIC = ["k_gram", "k_ip", "k_pw", "k_wapply", "k_h", "k_happly", "k_g", "k_gapply"]


def test_kernel_path_selection():
    """Uniform partitions with a compiled (N, K, M_l) set take the specialised kernels."""
    X, Q, g, W, H = _problem(4, 20, (4, 4, 4, 4), 5, 16, seed=1, fp32=True)
    assert plan(X, (4, 4, 4, 4), 5, 16, Q, g, W, H, True).kernel_names() == FAST
    X, Q, g, W, H = _problem(4, 20, (2, 3), 5, 16, seed=1, fp32=True)
    assert plan(X, (2, 3), 5, 16, Q, g, W, H, True).kernel_names() == GENERIC


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", STAGE_CASES, ids=lambda c: f"F{c[0]}T{c[1]}m{'x'.join(map(str, c[2]))}N{c[3]}K{c[4]}")
def test_one_step_parity_every_stage(case, fp32):
    F, T, mics, N, K = case
    X, Q, g, W, H = _problem(F, T, mics, N, K, seed=101, fp32=fp32)
    p = plan(X, mics, N, K, Q, g, W, H, fp32)
    for it in range(2):
        for stage in ("ip", "W", "H", "g"):
            before = state64(p)
            p.substep(stage)
            got = state64(p)
            want = oracle_stage(stage, X, mics, before)
            key = STAGE_KEY[stage]
            err = rel(got[key], want[key])
            tol = TOL_STAGE[fp32][key]
            if stage == "ip":
                kappa = _ip_condition(X, mics, before)
                tol = max(tol, (2e-8 if fp32 else 1e-15 * max(mics)) * kappa)
                if fp32:
                    c_got = D.nll(X, got["Q"], got["g"], got["W"], got["H"], mics)
                    c_want = D.nll(X, want["Q"], want["g"], want["W"], want["H"], mics)
                    c_tol = max(1e-6, 1e-9 * kappa)
                    assert abs(c_got - c_want) < c_tol * abs(c_want), (it, c_got, c_want, kappa)
            assert err < tol, (it, stage, err, tol)
            for other in ("Q", "g", "W", "H"):
                if other != key:
                    assert np.array_equal(got[other], before[other]), (stage, other)
    p.sync_status()


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(11, 333, (3, 2, 4), 3, 5), (13, 301, (4, 4, 4, 4), 5, 16), (6, 150, (16,), 5, 16)],
                         ids=["generic", "fast4x4", "fast16"])
def test_covariances_parity(fp32, shape):
    F, T, mics, N, K = shape
    X, Q, g, W, H = _problem(F, T, mics, N, K, seed=7, fp32=fp32)
    p = plan(X, mics, N, K, Q, g, W, H, fp32)
    V = p.covariances().cpu().numpy().astype(np.complex128)
    y = D.model_variance(D.source_psd(W, H), g)
    ref = D.weighted_covariances(X, y, mics)
    off = 0
    for l, ml in enumerate(mics):
        blk = V[:, off:off + ml ** 3].reshape(F, ml, ml, ml)
        assert rel(blk, ref[l]) < (2e-6 if fp32 else 1e-12), l
        off += ml ** 3


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_nll_and_separate_parity(fp32):
    F, T, mics, N, K = 13, 150, (2, 3), 3, 4
    X, Q, g, W, H = _problem(F, T, mics, N, K, seed=9, fp32=fp32)
    p = plan(X, mics, N, K, Q, g, W, H, fp32)
    ref = D.nll(X, Q, g, W, H, mics)
    assert nll_rel(p.nll(), ref, F, T, sum(mics)) < (1e-6 if fp32 else 1e-12)
    S = p.separate().cpu().numpy()
    Sref = D.separate(X, Q, g, W, H, mics)
    for n in range(N):
        assert rel(S[n], Sref[n]) < (1e-5 if fp32 else 1e-11), n


# ------------------------------------------------------------------ end to end, small_2x2 workload
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_end_to_end_small_2x2(fp32):
    w = synth.make("small_2x2")
    mics, N, K, it = w["mics"], w["N"], w["K"], w["iters"]
    X, Q, g, W, H = (as_precision(w[k], fp32) for k in ("X", "Q", "g", "W", "H"))
    p = plan(X, mics, N, K, Q, g, W, H, fp32)
    p.step(it)
    got = state64(p)
    ref = D.iterate(X, Q, g, W, H, mics, it)
    F, T, M = X.shape
    nref = D.nll(X, *ref, mics)
    ngot = p.nll()
    p.sync_status()
    if not fp32:
        for k, v in zip(("Q", "g", "W", "H"), ref):
            assert rel(got[k], v) < 1e-10, k
        assert nll_rel(ngot, nref, F, T, M) < 1e-12
    else:
        assert nll_rel(ngot, nref, F, T, M) < 1e-4
    S = p.separate().cpu().numpy()
    Sref = D.separate(X, *ref, mics)
    for n in range(N):
        assert rel(S[n], Sref[n]) < (1e-4 if fp32 else 1e-10), n


# ------------------------------------------------------------------ end to end, paper_4x4 workload
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_4x4_oracle.npz")
GOLDEN_TABLE2 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table2_oracle.npz")


def test_end_to_end_paper_4x4_fp32():
    """FP32 path at full size (F=513, T=625, four 4-mic subarrays, N=5, K=16), in the launch
    configuration bench.py times, against the oracle's stored trajectory on the same rounded
    inputs (tests/golden/make_golden.py): the cost at every checkpoint up to 100
    iterations and 8192 sampled entries of the separated images, 1e-4 relative per source."""
    ref = np.load(GOLDEN)
    w = synth.make("paper_4x4")
    mics, N, K = w["mics"], w["N"], w["K"]
    X, Q, g, W, H = (as_precision(w[k], True) for k in ("X", "Q", "g", "W", "H"))
    F, T, M = X.shape
    p = plan(X, mics, N, K, Q, g, W, H, True)
    assert p.kernel_names()[0] == "k_gramd_f"  # the specialised kernels bench.py times
    done = 0
    for c, cost in zip(ref["checkpoints"], ref["costs"]):
        p.step(int(c) - done)
        done = int(c)
        got = p.nll()
        assert nll_rel(got, cost, F, T, M) < 1e-4, (int(c), got, cost)
    p.sync_status()
    S = p.separate()
    idx = torch.as_tensor(ref["sample_index"].astype(np.int64), device=S.device)
    got = S[idx[0], idx[1], idx[2], idx[3]].cpu().numpy()
    want = ref["sample_values"]
    for n in range(N):
        sel = ref["sample_index"][0] == n
        assert rel(got[sel], want[sel]) < 1e-4, n


def test_end_to_end_table2_fp32():
    """FP32 path at the shape of the paper's Table II (F=2049, T=157, three 4-mic subarrays,
    N=3, K=16), where the H update runs split over the LDS windows of W, against the oracle's
    stored trajectory (tests/golden/make_golden.py): the cost at every checkpoint up to 50
    iterations and 8192 sampled entries of the separated images, 1e-4 relative per source."""
    ref = np.load(GOLDEN_TABLE2)
    w = synth.make("table2")
    mics, N, K = w["mics"], w["N"], w["K"]
    X, Q, g, W, H = (as_precision(w[k], True) for k in ("X", "Q", "g", "W", "H"))
    F, T, M = X.shape
    p = plan(X, mics, N, K, Q, g, W, H, True)
    names = p.kernel_names()
    assert names[0] == "k_gramd_f" and "k_hsum_f" in names and "k_hlam_f" in names, names
    done = 0
    for c, cost in zip(ref["checkpoints"], ref["costs"]):
        p.step(int(c) - done)
        done = int(c)
        got = p.nll()
        assert nll_rel(got, cost, F, T, M) < 1e-4, (int(c), got, cost)
    p.sync_status()
    S = p.separate()
    idx = torch.as_tensor(ref["sample_index"].astype(np.int64), device=S.device)
    got = S[idx[0], idx[1], idx[2], idx[3]].cpu().numpy()
    want = ref["sample_values"]
    for n in range(N):
        sel = ref["sample_index"][0] == n
        assert rel(got[sel], want[sel]) < 1e-4, n


# ------------------------------------------------------------------ invariants of the GPU result
def test_gpu_sweep_normalises_rows_and_cost_decreases():
    """After the IP stage mean_t P/y = 1 (eq. (16)); the cost never increases over stages (FP64)."""
    F, T, mics, N, K = 17, 210, (2, 2, 3), 3, 4
    X = synth.mixture(F, T, mics, N, K, 13)
    Q, g, W, H = synth.initial_state(F, T, mics, N, K, 14)
    p = plan(X, mics, N, K, Q, g, W, H, fp32=False)
    last = p.nll()
    for it in range(3):
        for stage in ("ip", "W", "H", "g"):
            if stage == "ip":
                s0 = state64(p)
            p.substep(stage)
            if stage == "ip":
                s1 = state64(p)
                y = D.model_variance(D.source_psd(s0["W"], s0["H"]), s0["g"])
                Pw = D.powers(X, s1["Q"], mics)
                np.testing.assert_allclose((Pw / y).mean(axis=1), 1.0, rtol=1e-10)
            cur = p.nll()
            assert cur <= last + 1e-9 * abs(last), (it, stage, cur, last)
            last = cur
    S = p.separate().cpu().numpy()
    assert rel(S.sum(axis=0), X) < 1e-11


def test_deterministic_and_resumable():
    F, T, mics, N, K = 21, 257, (4, 4, 4, 4), 5, 16
    X, Q, g, W, H = _problem(F, T, mics, N, K, seed=3, fp32=True, mixing="delay")
    a = plan(X, mics, N, K, Q, g, W, H, True).step(5)
    b = plan(X, mics, N, K, Q, g, W, H, True).step(3)
    b.step(2)
    sa, sb = a.state(), b.state()
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    assert a.nll() == b.nll()
    c = plan(X, mics, N, K, sa["Q"], sa["g"], sa["W"], sa["H"], True).step(2)
    d = a.step(2).state()
    for k, v in c.state().items():
        assert np.array_equal(v, d[k]), k


# ------------------------------------------------------------------ edge cases and error paths
@pytest.mark.parametrize("case", [
    (1, 5, (1,), 1, 1),          # smallest problem
    (2, 3, (1, 2), 1, 2),        # fewer frames than mics in total
    (3, 129, (2, 2), 2, 1),      # one slice plus one frame
    (2, 64, (1,) * 16, 4, 8),    # L = M: diagonal SCMs
    (4, 50, (16, 16, 16, 16), 3, 2),  # maximum mics
], ids=lambda c: f"F{c[0]}T{c[1]}L{len(c[2])}N{c[3]}K{c[4]}")
def test_edge_shapes_fp64(case):
    F, T, mics, N, K = case
    X, Q, g, W, H = _problem(F, T, mics, N, K, seed=5, fp32=False)
    p = plan(X, mics, N, K, Q, g, W, H, False)
    p.step(2)
    ref = D.iterate(X, Q, g, W, H, mics, 2)
    got = state64(p)
    for k, v in zip(("Q", "g", "W", "H"), ref):
        assert rel(got[k], v) < 1e-9, k
    assert nll_rel(p.nll(), D.nll(X, *ref, mics), F, T, sum(mics)) < 1e-11


def test_singular_system_is_reported():
    """A silent mic makes V singular; the oracle falls back to pinv, the GPU reports DFM_E_SINGULAR."""
    from paper_2605_19388_amd import DFMError
    F, T, mics, N, K = 3, 40, (2, 2), 2, 2
    X, Q, g, W, H = _problem(F, T, mics, N, K, seed=1, fp32=False)
    X[:, :, 1] = 0.0
    p = plan(X, mics, N, K, Q, g, W, H, False)
    p.substep("ip")
    with pytest.raises(DFMError) as e:
        p.sync_status()
    assert e.value.status == 6
    p.sync_status()  # cleared


def test_nonfinite_is_reported():
    from paper_2605_19388_amd import DFMError
    F, T, mics, N, K = 3, 40, (2, 2), 2, 2
    X, Q, g, W, H = _problem(F, T, mics, N, K, seed=2, fp32=True)
    W[0, 1, 0] = np.inf
    p = plan(X, mics, N, K, Q, g, W, H, True)
    p.step(1)
    with pytest.raises(DFMError) as e:
        p.sync_status()
    assert e.value.status in (5, 6)


def test_shape_errors_from_binding():
    from paper_2605_19388_amd import DFMError
    X, Q, g, W, H = _problem(3, 10, (2, 2), 2, 2, seed=1, fp32=True)
    with pytest.raises(DFMError):
        plan(X, (2, 3), 2, 2, Q, g, W, H, True)
