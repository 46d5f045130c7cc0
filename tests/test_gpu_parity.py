"""HIP path vs the FP64 oracle through the C ABI (GPU only).

One-step parity restarts the oracle from the GPU's own state before every stage,
so each kernel's error is measured alone; end-to-end parity runs both sides from
the same seeded inputs.  Every comparison is element by element:

* Q: per bin and subarray block, max |dQ| / max |Q_ref| over the block's entries
  (the rows of Q are defined only up to the block's scale);
* W, H, g (positive everywhere): max over entries of |d| / |ref|;
* covariances: per (f, l, mu) matrix, max |dV| / max |V_ref|;
* separated images: per source and per bin (see the end-to-end tests).

Each case prints the worst bin, its error and the condition number
kappa_fl = max over mu of max(cond(Q_fl V_flmu), cond(V_flmu)) there (the
amplification of input error by the solve of eq. (15), (Q V) b = e <=> V b = Q^-1 e).
Tolerances (every path sums V in FP64 from exact products):

* FP64: Q per block <= 1e-12 + 1e-15 kappa_fl (a backward-stable solve; kappa_fl
  measured by the oracle on the same inputs and required below 1e8); W, H, g <= 1e-12.
* FP32 (inputs and stored state in FP32, u = 6e-8): Q per block <= 2e-7 (the
  FP64 solve's output rounded to FP32 plus the FP32 weights 1/y; the measured
  worst is 8e-8 at kappa up to 7e7, independent of kappa); the cost after the
  sweep <= 1e-8 relative; W, H, g <= 2e-5 (FP32 sums of positive terms) for
  subarrays of up to 4 mics, 1e-4 for 16-mic blocks, where P = |q^H x|^2 in FP32
  loses up to u cond(Q_fl) on the faint rows of an ill-conditioned block.
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
from tests.gpu_common import (STAGE_KEY, announce, as_precision, elem_rel, nll_rel, oracle_stage,
                              per_bin_errors, plan, q_block_errors, rel, report, require_gpu, state64)
from tests.test_oracle_floors import faint_case, loud_case

pytestmark = pytest.mark.gpu

TOL_STAGE = {False: {"Q": 1e-12, "W": 1e-12, "H": 1e-12, "g": 1e-12},
             True: {"Q": 2e-7, "W": 2e-5, "H": 2e-5, "g": 2e-5}}
TOL_STAGE_FP32_16MIC = 1e-4   # W, H, g with 16-mic blocks (faint rows of ill-conditioned Q)
KAPPA_MAX = 1e8


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
    """kappa[f, l] = max over mu of cond(Q_fl V_flmu) and cond(V_flmu): the amplification of
    covariance errors in the solve of eq. (15), (Q V) b = e  <=>  V b = Q^{-1} e."""
    y = D.model_variance(D.source_psd(st["W"], st["H"]), st["g"])
    V = D.weighted_covariances(X, y, mics)
    Qb = D.q_blocks(st["Q"], mics)
    kappa = np.zeros((X.shape[0], len(mics)))
    for l in range(len(mics)):
        for mu in range(mics[l]):
            kappa[:, l] = np.maximum(kappa[:, l], np.maximum(np.linalg.cond(Qb[l] @ V[l][:, mu]),
                                                             np.linalg.cond(V[l][:, mu])))
    return kappa


def _stage_tol(key, fp32, mics):
    if fp32 and key != "Q" and max(mics) > 4:
        return TOL_STAGE_FP32_16MIC
    return TOL_STAGE[fp32][key]


def _check_stage(stage, X, mics, before, got, want, fp32, where):
    """Element-wise comparison of one stage's output with the oracle's; returns a report line."""
    key = STAGE_KEY[stage]
    if stage == "ip":
        err = q_block_errors(got["Q"], want["Q"], mics)
        kappa = _ip_condition(X, mics, before)
        assert kappa.max() < KAPPA_MAX, (where, kappa.max())
        tol = np.full_like(err, TOL_STAGE[True]["Q"]) if fp32 else 1e-12 + 1e-15 * kappa
        f, l = np.unravel_index(np.argmax(err / tol), err.shape)
        line = f"Q worst bin f={f} l={l}: {err[f, l]:.2e} (tol {tol[f, l]:.1e}, kappa {kappa[f, l]:.1e}; max kappa {kappa.max():.1e})"
        assert np.all(err <= tol), (where, line)
        if fp32:
            c_got = D.nll(X, got["Q"], got["g"], got["W"], got["H"], mics)
            c_want = D.nll(X, want["Q"], want["g"], want["W"], want["H"], mics)
            assert abs(c_got - c_want) <= 1e-8 * abs(c_want), (where, c_got, c_want)
        return line
    err = elem_rel(got[key], want[key])
    tol = _stage_tol(key, fp32, mics)
    assert err <= tol, (where, key, err, tol)
    return f"{key} {err:.1e} (tol {tol:.0e})"


# ------------------------------------------------------------------ one-step parity per stage
STAGE_CASES = [
    # (F, T, mics, N, K): several slices with a ragged tail, F not a multiple of the
    # 16-bin activation tiles.  Generic kernels: mixed or unlisted shapes.
    (37, 301, (2, 3, 1), 3, 4),
    (5, 260, (16,), 2, 3),
    (3, 40, (1, 1, 1, 1), 2, 2),
    # Subarrays of 5 to 12 mics: the IP sweep with the covariances inverted up front.
    (13, 140, (8, 3), 3, 4),
    (7, 157, (12,), 3, 16),
    (5, 90, (5, 7), 2, 3),
    # Shape-specialised kernels, one case per compiled (N, K, M_l) set.
    (9, 97, (4, 4, 4, 4), 5, 16),
    (37, 301, (4, 4, 4, 4), 5, 16),
    (18, 150, (16,), 5, 16),
    (20, 77, (4, 4), 3, 16),
    (20, 77, (4, 4, 4), 8, 16),
    (21, 50, (4, 4, 4), 3, 16),
    # Five to eight subarrays of 4 mics (M = 20-32): specialised in FP32; in FP64 only where a bin's
    # N x M values of g fit the FP64 covariance kernel's staging (N M <= 128), generic otherwise.
    (21, 120, (4,) * 6, 5, 16),
    (13, 90, (4,) * 8, 3, 16),
    (11, 70, (4,) * 5, 8, 16),
    (9, 64, (4,) * 7, 5, 16),
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
    # Eight 4-mic subarrays, N = 8: specialised in FP32, generic in FP64 (N M = 256 > 128).
    X, Q, g, W, H = _problem(4, 70, (4,) * 8, 8, 16, seed=1, fp32=True)
    assert plan(X, (4,) * 8, 8, 16, Q, g, W, H, True).kernel_names() == FAST
    X, Q, g, W, H = _problem(4, 70, (4,) * 8, 8, 16, seed=1, fp32=False)
    assert plan(X, (4,) * 8, 8, 16, Q, g, W, H, False).kernel_names() == GENERIC


def _run_stages(X, Q, g, W, H, mics, N, K, fp32, iters, where):
    p = plan(X, mics, N, K, Q, g, W, H, fp32)
    for it in range(iters):
        lines = []
        for stage in ("ip", "W", "H", "g"):
            before = state64(p)
            p.substep(stage)
            got = state64(p)
            want = oracle_stage(stage, X, mics, before)
            lines.append(_check_stage(stage, X, mics, before, got, want, fp32, (where, it, stage)))
            for other in ("Q", "g", "W", "H"):
                if other != STAGE_KEY[stage]:
                    assert np.array_equal(got[other], before[other]), (stage, other)
        report(f"{where} it{it}: " + "; ".join(lines))
    p.sync_status()


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", STAGE_CASES, ids=lambda c: f"F{c[0]}T{c[1]}m{'x'.join(map(str, c[2]))}N{c[3]}K{c[4]}")
def test_one_step_parity_every_stage(case, fp32):
    F, T, mics, N, K = case
    X, Q, g, W, H = _problem(F, T, mics, N, K, seed=101, fp32=fp32)
    _run_stages(X, Q, g, W, H, mics, N, K, fp32, 2, f"{case} {'fp32' if fp32 else 'fp64'}")


# Floors of Sec. IV-A active: a faint recording with a tiny model (the model variance floored at
# every (f, t, m); in FP64 every MM denominator as well), and a loud recording (every IP
# normaliser b^H V b floored).  FP64 runs two iterations; FP32 one, since a second floored
# iteration shrinks lambda = W H below FP32's normal range (the oracle's FP64 does not).
FLOOR_SHAPES = [((3,), 5, 40, 2, 2), ((2, 2), 7, 50, 2, 4), ((4, 4, 4, 4), 9, 97, 5, 16), ((16,), 5, 60, 5, 16)]


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["faint", "loud"])
@pytest.mark.parametrize("shape", FLOOR_SHAPES, ids=lambda c: "x".join(map(str, c[0])))
def test_one_step_parity_floors_active(shape, kind, fp32):
    mics, F, T, N, K = shape
    X, Q, g, W, H = (faint_case if kind == "faint" else loud_case)(mics, F=F, T=T, N=N, K=K)
    X, Q, g, W, H = (as_precision(a, fp32) for a in (X, Q, g, W, H))
    y = D.model_variance(D.source_psd(W, H), g)
    if kind == "faint":
        assert np.all(y == D.EPS)  # floored everywhere
    else:
        V = D.weighted_covariances(X, y, mics)
        Ql = D.q_blocks(Q, mics)[0]
        b = np.linalg.solve(Ql @ V[0][:, 0], np.eye(mics[0])[:, 0])
        floored = np.einsum("fa,fab,fb->f", b.conj(), V[0][:, 0], b).real < D.EPS
        report(f"loud{mics}: first-row normaliser floored in {int(floored.sum())} of {F} bins")
        assert floored.any()
    _run_stages(X, Q, g, W, H, mics, N, K, fp32, 1 if fp32 else 2, f"{kind}{shape[0]} {'fp32' if fp32 else 'fp64'}")


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
    tol = 5e-7 if fp32 else 1e-13  # FP32: the weights 1/y (one rounding each); FP64: summation order
    for l, ml in enumerate(mics):
        blk = V[:, off:off + ml ** 3].reshape(F, ml, ml, ml)
        err = per_bin_errors(blk, ref[l], axes=(2, 3))  # [F, mu]: one value per matrix V_flmu
        f, mu = np.unravel_index(np.argmax(err), err.shape)
        report(f"covariances {shape} {'fp32' if fp32 else 'fp64'} l={l}: worst f={f} mu={mu} {err[f, mu]:.2e}")
        assert err.max() <= tol, (l, f, mu, err.max())
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
    _check_images(S, Sref, X, 1e-5 if fp32 else 1e-11, f"one-shot {'fp32' if fp32 else 'fp64'}")


def _check_images(S, Sref, X, tol, where):
    """Separated images element by element: per source over every bin, ||dS_n|| / ||S_n|| <= tol
    (the bar of the method), and per (source, bin) max |dS_nf| / max |x_f| <= tol (the images of
    one bin sum to its mixture, so this is each bin's error on the bin's own scale)."""
    N = S.shape[0]
    for n in range(N):
        e = rel(S[n], Sref[n])
        assert e <= tol, (where, n, e)
    xs = np.abs(X).max(axis=(1, 2))                                 # [F]
    eb = np.abs(S - Sref).max(axis=(2, 3)) / xs[None, :]            # [N, F]
    n, f = np.unravel_index(np.argmax(eb), eb.shape)
    src = max(rel(S[k], Sref[k]) for k in range(N))
    report(f"{where}: images worst source {src:.2e}; worst bin n={n} f={f} {eb[n, f]:.2e}")
    assert eb.max() <= tol, (where, n, f, eb.max())


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
    _check_images(S, Sref, X, 1e-4 if fp32 else 1e-10, f"small_2x2 {'fp32' if fp32 else 'fp64'}")


# ------------------------------------------------------------------ end to end at full size
GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _end_to_end_golden(name, expect_kernels):
    """FP32 path at full size, in the launch configuration bench.py times, against the oracle's
    stored trajectory on the same rounded inputs (tests/golden/make_golden.py): the cost at every
    checkpoint, and the separated images over every entry, formed by the oracle from its stored
    final state, 1e-4 relative per source and per bin."""
    ref = np.load(os.path.join(GOLDEN_DIR, f"{name}_oracle.npz"))
    w = synth.make(name)
    mics, N, K = w["mics"], w["N"], w["K"]
    X, Q, g, W, H = (as_precision(w[k], True) for k in ("X", "Q", "g", "W", "H"))
    F, T, M = X.shape
    p = plan(X, mics, N, K, Q, g, W, H, True)
    names = p.kernel_names()
    for k in expect_kernels:
        assert k in names, (k, names)
    done = 0
    for c, cost in zip(ref["checkpoints"], ref["costs"]):
        p.step(int(c) - done)
        done = int(c)
        got = p.nll()
        e = nll_rel(got, cost, F, T, M)
        report(f"{name} iteration {int(c)}: cost {got:.10e} oracle {cost:.10e} rel {e:.1e}")
        assert e < 1e-4, (int(c), got, cost)
    p.sync_status()
    assert done == int(ref["final_iteration"])
    S = p.separate()
    # The stored samples (drawn at fixed positions) first, then every entry.
    idx = torch.as_tensor(ref["sample_index"].astype(np.int64), device=S.device)
    got = S[idx[0], idx[1], idx[2], idx[3]].cpu().numpy()
    for n in range(N):
        sel = ref["sample_index"][0] == n
        assert rel(got[sel], ref["sample_values"][sel]) < 1e-4, n
    S = S.cpu().numpy()
    Sref = D.separate(X, ref["Q"], ref["g"], ref["W"], ref["H"], mics)
    assert np.array_equal(Sref[idx[0].cpu().numpy(), idx[1].cpu().numpy(), idx[2].cpu().numpy(),
                               idx[3].cpu().numpy()], ref["sample_values"])  # the stored state is the run's
    _check_images(S, Sref, X, 1e-4, name)


def test_end_to_end_paper_4x4_fp32():
    """F=513, T=625, four 4-mic subarrays, N=5, K=16, 100 iterations (the bench workload)."""
    _end_to_end_golden("paper_4x4", ["k_gramd_f"])


def test_end_to_end_table2_fp32():
    """The shape of the paper's Table II (F=2049, T=157, three 4-mic subarrays, N=3, K=16), 50
    iterations; W[n] spans several LDS windows, so the H update runs split over the bins."""
    _end_to_end_golden("table2", ["k_gramd_f", "k_hsum_f", "k_hlam_f"])


def test_end_to_end_paper_16_fp32():
    """The conventional method on the paper_4x4 recording: one 16-mic block (L = 1), 100
    iterations; the 16 x 16 covariances on the FP64 matrix cores and the generic IP sweep."""
    _end_to_end_golden("paper_16", ["k_gram_f", "k_ip"])


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
    assert q_block_errors(got["Q"], ref[0], mics).max() < 1e-9
    for k, v in zip(("g", "W", "H"), ref[1:]):
        assert elem_rel(got[k], v) < 1e-9, k
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
    from paper_2605_19388_amd import binding
    p = plan(X, mics, N, K, Q, g, W, H, True, flags=binding.F_CHECK_FINITE)
    p.step(1)
    with pytest.raises(DFMError) as e:
        p.sync_status()
    assert e.value.status in (5, 6)


def test_shape_errors_from_binding():
    from paper_2605_19388_amd import DFMError
    X, Q, g, W, H = _problem(3, 10, (2, 2), 2, 2, seed=1, fp32=True)
    with pytest.raises(DFMError):
        plan(X, (2, 3), 2, 2, Q, g, W, H, True)
