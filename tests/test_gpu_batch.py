"""Batches of uneven mixtures (dfm_batch_*), the tile parameter and the autotuner on the GPU,
through the C ABI (GPU only).  A batch replays graphs in which every plan is a branch; each plan's
state must equal, bit for bit, a twin plan stepped alone with dfm_step."""
import numpy as np
import pytest
import torch

from oracle import dfmnmf as D
from paper_2605_19388_amd import autotune, binding, synth
from tests.gpu_common import announce, as_precision, nll_rel, plan, report, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu(request):
    require_gpu()
    announce(request.node.nodeid)
    yield
    torch.cuda.synchronize()


# Uneven shapes: 2-5 subarrays of 4 mics, N in {3, 5, 8}, T from 40 to 201; specialised sets and
# the generic kernels (five subarrays; one 2-mic partition); FP32 and FP64; several tiles.
SHAPES = [(17, 40, (4, 4), 3, 16, True, 0), (17, 77, (4, 4, 4), 8, 16, True, 32),
          (17, 130, (4, 4, 4, 4), 5, 16, True, 64), (17, 201, (4,) * 5, 3, 16, True, 0),
          (17, 96, (4, 4, 4, 4), 8, 16, False, 16), (17, 150, (2, 3), 3, 4, True, 0)]


def _plan(i, shape):
    F, T, mics, N, K, fp32, tile = shape
    X = synth.mixture(F, T, mics, N, K, 100 + i, mixing="delay")
    Q, g, W, H = synth.initial_state(F, T, mics, N, K, 200 + i)
    X, Q, g, W, H = (as_precision(a, fp32) for a in (X, Q, g, W, H))
    cdt, rdt = (np.complex64, np.float32) if fp32 else (np.complex128, np.float64)
    return binding.DistributedFastMNMF(X.astype(cdt), mics, N, K, W=W.astype(rdt), H=H.astype(rdt),
                                       Q=Q.astype(cdt), g=g.astype(rdt), tile=tile)


def test_batch_equals_unbatched():
    a = [_plan(i, s) for i, s in enumerate(SHAPES)]
    b = [_plan(i, s) for i, s in enumerate(SHAPES)]
    batch = binding.Batch(a)
    for n in (1, 9, 3, 17):   # first iteration alone, with the group-of-eight graph, singles
        batch.step(n)
        for p in b:
            p.step(n)
        costs = [p.nll() for p in a]   # eager work between replays
        torch.cuda.synchronize()
        for i, (pa, pb) in enumerate(zip(a, b)):
            sa, sb = pa.state(), pb.state()
            for k in sa:
                assert np.array_equal(sa[k], sb[k]), (n, i, k)
            assert costs[i] == pb.nll()
    for p in a + b:
        p.sync_status()
    batch.close()


@pytest.mark.parametrize("shape", [(33, 301, (4, 4, 4, 4), 5, 16), (20, 250, (2, 3, 1), 3, 4)],
                         ids=["fast", "generic"])
def test_tiles_keep_the_result(shape):
    """Every tile gives the oracle's trajectory to the FP32 bar (3 iterations)."""
    F, T, mics, N, K = shape
    X = as_precision(synth.mixture(F, T, mics, N, K, 3, mixing="delay"), True)
    Q, g, W, H = (as_precision(a, True) for a in synth.initial_state(F, T, mics, N, K, 4))
    ref = D.nll(X, *D.iterate(X, Q, g, W, H, mics, 3), mics)
    for tile in autotune.CANDIDATES:
        p = binding.DistributedFastMNMF(X.astype(np.complex64), mics, N, K, W=W.astype(np.float32),
                                        H=H.astype(np.float32), Q=Q.astype(np.complex64), g=g.astype(np.float32),
                                        tile=tile)
        p.step(3)
        e = nll_rel(p.nll(), ref, F, T, sum(mics))
        report(f"tile {tile} {shape}: cost rel error {e:.1e}")
        assert e < 1e-6


def test_autotuner_picks_a_measured_candidate():
    best, timings = autotune.tune(65, 420, (4, 4, 4, 4), 5, 16, iters=2, reps=1)
    report(f"autotune (65, 420, 4x4x4x4, 5, 16): {best} from " + ", ".join(f"{c}: {t:.3f} ms" for c, t in timings.items()))
    assert best in autotune.CANDIDATES and set(timings) == set(autotune.CANDIDATES)
    again, t2 = autotune.tune(65, 430, (4, 4, 4, 4), 5, 16)   # same shape class: cached
    assert again == best and t2 == {}


def test_batch_argument_errors():
    p = _plan(0, SHAPES[0])
    lib = binding.load()
    import ctypes
    out = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 2)(p._plan.value, p._plan.value)
    assert lib.dfm_batch_create(ctypes.byref(out), arr, 2) == 1      # the same plan twice
    assert lib.dfm_batch_create(ctypes.byref(out), arr, 0) == 1
    assert lib.dfm_batch_step(None, 1, None) == 1
