"""BF16 covariances (DFM_F_GRAM_BF16): eq. (14) from BF16 operands on the matrix cores with FP32
sums, the IP solves in FP64, against the FP64 oracle (GPU only; through the C ABI).

The error of this form is stated, not hidden: each term w x_a conj(x_b) of eq. (14) is formed
from the BF16 roundings of w x_a and x_b (relative error up to 2^-9 each), so a covariance entry
is off by up to about 2^-8 of the sum of its terms' magnitudes.  The tests hold the covariances
to that bound and report the cost and separated-image errors of a full run against the oracle's
FP64 trajectory, holding them to the bounds measured for this form (below)."""
import os

import numpy as np
import pytest
import torch

from oracle import dfmnmf as D
from paper_2605_19388_amd import binding, synth
from tests.common import random_state
from tests.gpu_common import announce, as_precision, nll_rel, plan, rel, report, require_gpu

pytestmark = pytest.mark.gpu

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(autouse=True)
def _gpu(request):
    require_gpu()
    announce(request.node.nodeid)
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("shape", [(13, 301, (4, 4, 4, 4), 5, 16), (20, 77, (4, 4, 4), 3, 16),
                                   (9, 80, (2, 2), 2, 4), (11, 150, (4, 4), 3, 16)],
                         ids=["4x4x4x4", "4x4x4", "2x2", "4x4"])
def test_bf16_covariances_within_rounding_bound(shape):
    """Every entry of every V_flmu within 2^-7 of the sum of its terms' magnitudes
    (sum_t w |x_a| |x_b|, at most sqrt(V_aa V_bb) after the 1/T) -- twice the rounding bound."""
    F, T, mics, N, K = shape
    X = as_precision(synth.mixture(F, T, mics, N, K, 7, mixing="delay"), True)
    Q, g, W, H = (as_precision(a, True) for a in random_state(F, T, mics, N, K, 8))
    p = plan(X, mics, N, K, Q, g, W, H, True, flags=binding.F_GRAM_BF16)
    assert p.kernel_names()[0] == "k_gramb_f"
    V = p.covariances().cpu().numpy().astype(np.complex128)
    y = D.model_variance(D.source_psd(W, H), g)
    ref = D.weighted_covariances(X, y, mics)
    off, worst = 0, 0.0
    for l, ml in enumerate(mics):
        blk = V[:, off:off + ml ** 3].reshape(F, ml, ml, ml)      # [f, mu, a, b]
        d = np.sqrt(np.abs(np.einsum("fmaa->fma", ref[l].real)))  # sqrt(V_aa) per (f, mu)
        scale = d[:, :, :, None] * d[:, :, None, :]
        err = np.abs(blk - ref[l]) / scale
        worst = max(worst, float(err.max()))
        off += ml ** 3
    report(f"bf16 covariances {shape}: worst |dV_ab| / sqrt(V_aa V_bb) = {worst:.2e} (bound {2.0 ** -7:.1e})")
    assert worst <= 2.0 ** -7


# This form against the FP64 oracle's trajectory at paper_4x4 (F=513, T=625, 4 x 4 mics, N=5, K=16,
# 100 iterations, the same FP32-rounded inputs), measured on MI355X: the cost within 1e-5 at every
# checkpoint, so it meets the 1e-4 bar of the method; the separated images 1.4e-2 to 1.9e-2 per
# source, so they miss it (the BF16 rounding of every term moves Q's weakly determined rows, which
# the cost barely sees).  The bounds are the cost bar and the images' measured error with margin.
BF16_COST_TOL = 1e-4
BF16_IMAGE_TOL = 5e-2


def test_bf16_end_to_end_paper_4x4_error_stated():
    ref = np.load(os.path.join(GOLDEN_DIR, "paper_4x4_oracle.npz"))
    w = synth.make("paper_4x4")
    mics, N, K = w["mics"], w["N"], w["K"]
    X, Q, g, W, H = (as_precision(w[k], True) for k in ("X", "Q", "g", "W", "H"))
    F, T, M = X.shape
    p = plan(X, mics, N, K, Q, g, W, H, True, flags=binding.F_GRAM_BF16)
    assert p.kernel_names()[0] == "k_gramb_f"
    done, worst_cost = 0, 0.0
    for c, cost in zip(ref["checkpoints"], ref["costs"]):
        p.step(int(c) - done)
        done = int(c)
        e = nll_rel(p.nll(), cost, F, T, M)
        worst_cost = max(worst_cost, e)
        report(f"bf16 paper_4x4 iteration {int(c)}: cost rel error {e:.2e}")
    p.sync_status()
    S = p.separate().cpu().numpy()
    Sref = D.separate(X, ref["Q"], ref["g"], ref["W"], ref["H"], mics)
    errs = [rel(S[n], Sref[n]) for n in range(N)]
    report(f"bf16 paper_4x4: worst cost error {worst_cost:.2e}; separated images per source " +
           ", ".join(f"{e:.2e}" for e in errs))
    assert worst_cost <= BF16_COST_TOL
    assert max(errs) <= BF16_IMAGE_TOL
