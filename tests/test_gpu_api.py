"""The C ABI's launch options on the GPU: graph replays, the cost trace, the finite check and
the largest subarrays (GPU only; every call goes through the C ABI)."""
import numpy as np
import pytest
import torch

from oracle import dfmnmf as D
from paper_2605_19388_amd import binding, synth
from tests.common import random_state
from tests.gpu_common import announce, as_precision, nll_rel, plan, rel, require_gpu, state64

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu(request):
    require_gpu()
    announce(request.node.nodeid)
    yield
    torch.cuda.synchronize()


def _problem(F, T, mics, N, K, seed, fp32, mixing="iid"):
    X = synth.mixture(F, T, mics, N, K, seed, mixing=mixing)
    Q, g, W, H = random_state(F, T, mics, N, K, seed + 1)
    return tuple(as_precision(a, fp32) for a in (X, Q, g, W, H))


def _same_state(a, b):
    sa, sb = a.state(), b.state()
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k


CASES = [((21, 257, (4, 4, 4, 4), 5, 16), True), ((13, 150, (2, 3), 3, 4), True), ((9, 80, (2, 2), 2, 4), False)]


@pytest.mark.parametrize("case,fp32", CASES, ids=["fast4x4", "generic", "fast2x2_fp64"])
def test_graph_replays_equal_plain_launches(case, fp32):
    """dfm_step replays captured graphs (the first iteration, later ones, batches of eight); the
    same plan made with DFM_F_NO_GRAPH launches every kernel plainly.  Both must agree bit for bit
    after every call, with the program's own eager work (cost, synchronisation) between replays."""
    F, T, mics, N, K = case
    X, Q, g, W, H = _problem(F, T, mics, N, K, seed=31, fp32=fp32, mixing="delay")
    a = plan(X, mics, N, K, Q, g, W, H, fp32)
    b = plan(X, mics, N, K, Q, g, W, H, fp32, flags=binding.F_NO_GRAPH)
    for n in (1, 9, 3, 17, 1, 2):  # graph[0] alone, with the batch graph, with single later ones
        a.step(n)
        b.step(n)
        assert a.nll() == b.nll(), n
        torch.cuda.synchronize()
        _same_state(a, b)
    a.sync_status()
    b.sync_status()


@pytest.mark.parametrize("case,fp32", CASES, ids=["fast4x4", "generic", "fast2x2_fp64"])
def test_cost_trace_records_every_iteration(case, fp32):
    """DFM_F_TRACE_NLL: the cost after each iteration of one dfm_step call equals dfm_nll after
    each of the same number of one-iteration calls (the same kernels, so bit for bit), and the
    state after the call equals the untraced run's."""
    F, T, mics, N, K = case
    X, Q, g, W, H = _problem(F, T, mics, N, K, seed=41, fp32=fp32, mixing="delay")
    a = plan(X, mics, N, K, Q, g, W, H, fp32, flags=binding.F_TRACE_NLL)
    b = plan(X, mics, N, K, Q, g, W, H, fp32)
    a.step(12)
    want = []
    for _ in range(12):
        b.step(1)
        want.append(b.nll())
    got, n = a.nll_trace()
    assert n == 12 and len(got) == 12
    np.testing.assert_array_equal(got, np.array(want))
    _same_state(a, b)
    a.step(3)
    got, n = a.nll_trace()
    assert n == 15 and got[-1] == a.nll()


def test_cost_trace_decreases_fp64():
    """The traced costs of an FP64 run never increase (every update of the method is a
    majorisation-minimisation or exact coordinate step) and match the oracle's."""
    F, T, mics, N, K = 17, 210, (2, 2, 3), 3, 4
    X = synth.mixture(F, T, mics, N, K, 13)
    Q, g, W, H = synth.initial_state(F, T, mics, N, K, 14)
    p = plan(X, mics, N, K, Q, g, W, H, fp32=False, flags=binding.F_TRACE_NLL)
    p.step(6)
    got, n = p.nll_trace()
    assert n == 6
    assert np.all(np.diff(got) <= 1e-9 * np.abs(got[1:]))
    want = []
    st = (Q, g, W, H)
    for _ in range(6):
        st = D.iterate(X, *st, mics, 1)
        want.append(D.nll(X, *st, mics))
    for c, r in zip(got, want):
        assert nll_rel(c, r, F, T, sum(mics)) < 1e-11


def test_trace_call_needs_the_flag():
    X, Q, g, W, H = _problem(3, 10, (2, 2), 2, 2, seed=1, fp32=True)
    p = plan(X, (2, 2), 2, 2, Q, g, W, H, True)
    with pytest.raises(binding.DFMError) as e:
        p.nll_trace()
    assert e.value.status == 1


@pytest.mark.parametrize("flags,expect", [(binding.F_CHECK_FINITE, True), (0, False)], ids=["check", "nocheck"])
def test_finite_check_flag(flags, expect):
    """A non-finite parameter is reported as DFM_E_NONFINITE only with DFM_F_CHECK_FINITE."""
    F, T, mics, N, K = 3, 40, (2, 2), 2, 2
    X, Q, g, W, H = _problem(F, T, mics, N, K, seed=2, fp32=True)
    W[0, 1, 0] = np.inf
    p = plan(X, mics, N, K, Q, g, W, H, True, flags=flags)
    p.step(1)
    status = 0
    try:
        p.sync_status()
    except binding.DFMError as e:
        status = e.status
    if expect:
        assert status in (5, 6)
    else:
        assert status != 5


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
@pytest.mark.parametrize("mics", [(32,), (32, 32), (32, 5)], ids=["32", "32x32", "32x5"])
def test_largest_subarrays(mics, fp32):
    """Subarrays of up to 32 mics (the generic kernels), two iterations against the oracle."""
    F, T, N, K = 3, 90, 3, 2
    X, Q, g, W, H = _problem(F, T, mics, N, K, seed=9, fp32=fp32)
    p = plan(X, mics, N, K, Q, g, W, H, fp32)
    p.step(2)
    ref = D.iterate(X, Q, g, W, H, mics, 2)
    got = state64(p)
    tol = 1e-4 if fp32 else 1e-9
    for k, v in zip(("Q", "g", "W", "H"), ref):
        assert rel(got[k], v) < tol, k
    assert nll_rel(p.nll(), D.nll(X, *ref, mics), F, T, sum(mics)) < (1e-5 if fp32 else 1e-11)
    p.sync_status()
