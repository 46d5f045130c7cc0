"""dfm_run_noalloc (the entry point that allocates nothing: its workspace is the library's static
device array) against the plan-based entry points dfm_init + dfm_step + dfm_nll on the same inputs
(GPU only; through the C ABI).  Two calls in a row, the second on a smaller input, must each equal
the plan's result bit for bit (the same kernels on the same inputs)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2605_19388_amd import binding, synth
from tests.common import random_state
from tests.gpu_common import announce, as_precision, plan, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu(request):
    require_gpu()
    announce(request.node.nodeid)
    yield
    torch.cuda.synchronize()


def _inputs(F, T, mics, N, K, seed, fp32):
    X = synth.mixture(F, T, mics, N, K, seed, mixing="delay")
    Q, g, W, H = random_state(F, T, mics, N, K, seed + 1)
    return tuple(as_precision(a, fp32) for a in (X, Q, g, W, H))


def _noalloc(X, Q, g, W, H, mics, N, K, n_iter, fp32, flags=0):
    lib = binding.load()
    dev = torch.device("cuda:0")
    cdt, rdt = (torch.complex64, torch.float32) if fp32 else (torch.complex128, torch.float64)
    t = {k: torch.as_tensor(v).to(device=dev, dtype=cdt if np.iscomplexobj(v) else rdt).contiguous()
         for k, v in (("X", X), ("Q", Q), ("g", g), ("W", W), ("H", H))}
    cost = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    status = torch.full((1,), -1, dtype=torch.int32, device=dev)
    F, T, M = X.shape
    prob = binding.make_problem(F, T, mics, N, K, binding.DFM_C64 if fp32 else binding.DFM_C128, 1e-6, flags)
    st = lib.dfm_run_noalloc(ctypes.byref(prob), t["X"].data_ptr(), t["Q"].data_ptr(), t["g"].data_ptr(),
                             t["W"].data_ptr(), t["H"].data_ptr(), int(n_iter), cost.data_ptr(), status.data_ptr(),
                             torch.cuda.current_stream(dev).cuda_stream)
    torch.cuda.synchronize()
    state = {k: t[k].cpu().numpy() for k in ("Q", "g", "W", "H")}
    return st, state, float(cost.item()), int(status.item())


def _compare(case, n_iter, fp32):
    F, T, mics, N, K = case
    X, Q, g, W, H = _inputs(F, T, mics, N, K, seed=F + T, fp32=fp32)
    st, got, cost, status = _noalloc(X, Q, g, W, H, mics, N, K, n_iter, fp32)
    assert st == 0 and status == 0, (st, status)
    p = plan(X, mics, N, K, Q, g, W, H, fp32)
    p.step(n_iter)
    want_cost = p.nll()
    want = p.state()
    for k in want:
        assert np.array_equal(got[k], want[k]), (case, k)
    assert cost == want_cost, (case, cost, want_cost)
    return cost


def test_noalloc_equals_plan_on_two_calls_second_smaller():
    """Paper-shaped partition first, then a smaller problem: the static array keeps the first
    call's contents, which the second call must not read."""
    c1 = _compare((40, 300, (4, 4, 4, 4), 5, 16), 5, True)
    c2 = _compare((13, 77, (2, 2), 2, 4), 4, True)
    c3 = _compare((9, 50, (2, 3), 3, 4), 3, False)   # generic kernels, FP64
    assert np.isfinite([c1, c2, c3]).all()


def test_noalloc_full_size_workload_and_limit():
    """paper_4x4 at full size fits the static array; a problem whose workspace exceeds it is
    refused before anything is launched (DFM_E_WORKSPACE)."""
    w = synth.make("paper_4x4")
    X, Q, g, W, H = (as_precision(w[k], True) for k in ("X", "Q", "g", "W", "H"))
    st, got, cost, status = _noalloc(X, Q, g, W, H, w["mics"], w["N"], w["K"], 3, True)
    assert st == 0 and status == 0
    p = plan(X, w["mics"], w["N"], w["K"], Q, g, W, H, True)
    p.step(3)
    assert cost == p.nll()
    for k, v in p.state().items():
        assert np.array_equal(got[k], v), k
    lib = binding.load()
    big = binding.make_problem(513, 625, (16,), 5, 16, binding.DFM_C64)
    assert binding.workspace_size(big) > binding.NOALLOC_SCRATCH_BYTES
    fake = ctypes.c_void_p(0x1000)
    assert lib.dfm_run_noalloc(ctypes.byref(big), fake, fake, fake, fake, fake, 1, None, None, None) == 3
    traced = binding.make_problem(5, 9, (2, 2), 2, 2, binding.DFM_C64, 1e-6, binding.F_TRACE_NLL)
    assert lib.dfm_run_noalloc(ctypes.byref(traced), fake, fake, fake, fake, fake, 1, None, None, None) == 1
