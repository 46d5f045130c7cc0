"""Initial parameters from source-image estimates (Sec. IV-A, steps 3, 5, 6) on the GPU against
the oracle (oracle/init.py), through the C ABI (GPU only).

Q is compared per bin and subarray block, element by element relative to the block's largest
entry; g and h entry by entry.  Both sides work in FP64, so the differences are rounding
amplified by the conditioning of each step, which every case reports: the eigenvectors of step 5
move by about u cond(B_fl) (1 + 1 / gap_fl), with B_fl = R_f,N^(l) (its Cholesky factor maps the
pencil to a Hermitian matrix) and gap_fl the smallest relative gap between its generalized
eigenvalues; g inherits the same; h = c^H R^-1 c moves by about u cond(R_fn).  Bounds: Q_fl <=
1e-15 cond(B_fl) (1 + 1 / gap_fl), g <= its largest such value, h <= 1e-15 max cond(R_fn), each
plus 2e-7 when the outputs are rounded to FP32 (complex64 images)."""
import numpy as np
import pytest
import torch

from oracle import dfmnmf as D
from oracle import init as I
from paper_2605_19388_amd import binding, synth
from tests.gpu_common import announce, as_precision, nll_rel, plan, q_block_errors, report, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu(request):
    require_gpu()
    announce(request.node.nodeid)
    yield
    torch.cuda.synchronize()


def _conditioning(R, mics):
    """Per (f, l): cond(B_fl) and the smallest relative gap between consecutive generalized
    eigenvalues of the pencil (R_f,N-1^(l), R_f,N^(l)) (inf for one mic)."""
    F, N = R.shape[:2]
    gaps = np.full((F, len(mics)), np.inf)
    kb = np.ones((F, len(mics)))
    for l, (ml, (mo, _)) in enumerate(zip(mics, D.block_offsets(mics))):
        sl = slice(mo, mo + ml)
        for f in range(F):
            kb[f, l] = np.linalg.cond(R[f, N - 1, sl, sl])
            _, lam = I.joint_diagonaliser(R[f, N - 2, sl, sl], R[f, N - 1, sl, sl])
            if ml > 1:
                gaps[f, l] = np.min(np.diff(lam) / np.maximum(np.abs(lam[1:]), np.abs(lam[:-1])))
    return kb, gaps


CASES = [((9, 120, (4, 4, 4, 4), 5, 16), "delay"), ((13, 200, (2, 3, 1), 3, 4), "iid"),
         ((5, 90, (16,), 5, 8), "delay"), ((4, 300, (8, 8), 2, 4), "iid"), ((3, 60, (1, 1), 2, 2), "iid")]


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case,mixing", CASES, ids=lambda c: "x".join(map(str, c[2])) if isinstance(c, tuple) else c)
def test_initialise_matches_oracle(case, mixing, fp32):
    F, T, mics, N, K = case
    _, C = synth.source_images(F, T, mics, N, K, seed=F + T, mixing=mixing)
    C = as_precision(C, fp32)
    Qg, gg, hg = binding.initialise(C.astype(np.complex64 if fp32 else np.complex128), mics)
    Qg, gg, hg = (t.cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64) for t in (Qg, gg, hg))
    R = I.image_covariances(C)
    Q, g, h = I.initialise(C, mics)
    kb, gap = _conditioning(R, mics)
    kr = max(np.linalg.cond(R[f, n]) for f in range(F) for n in range(N))
    out = 2e-7 if fp32 else 0.0
    amp = kb * (1.0 + 1.0 / gap)
    tol = out + 1e-15 * amp
    eq = q_block_errors(Qg, Q, mics)
    f, l = np.unravel_index(np.argmax(eq / tol), eq.shape)
    eg = float(np.max(np.abs(gg - g) / np.abs(g)))
    eh = float(np.max(np.abs(hg - h) / np.abs(h)))
    tg, th = out + 1e-15 * amp.max(), out + 1e-15 * kr
    report(f"initialise {case} {'fp32' if fp32 else 'fp64'}: Q worst f={f} l={l} {eq[f, l]:.2e} (tol {tol[f, l]:.1e}: "
           f"cond(B) {kb[f, l]:.1e}, gap {gap[f, l]:.1e}); g {eg:.1e} (tol {tg:.1e}); h {eh:.1e} (tol {th:.1e}, "
           f"cond(R) {kr:.1e})")
    assert np.all(eq <= tol), (f, l, eq[f, l], tol[f, l])
    assert eg <= tg
    assert eh <= th


def test_initialise_then_iterate_fp64():
    """The GPU's initial state runs the method from there exactly as the oracle's does: ten
    iterations from each, costs within 1e-10."""
    F, T, mics, N, K = 11, 150, (4, 4, 4, 4), 5, 16
    X, C = synth.source_images(F, T, mics, N, K, seed=3, mixing="delay")
    Qg, gg, _ = binding.initialise(C, mics, with_h=False)
    Q, g, _ = I.initialise(C, mics)
    _, _, W, H = synth.initial_state(F, T, mics, N, K, seed=4)
    p = plan(X, mics, N, K, Qg.cpu().numpy(), gg.cpu().numpy(), W, H, fp32=False)
    p.step(10)
    ref = D.iterate(X, Q, g, W, H, mics, 10)
    e = nll_rel(p.nll(), D.nll(X, *ref, mics), F, T, sum(mics))
    report(f"initialise + 10 iterations fp64: cost rel error {e:.1e}")
    assert e < 1e-10


def test_initialise_argument_errors():
    lib = binding.load()
    import ctypes
    one = binding.make_problem(3, 10, (2, 2), 1, 2, binding.DFM_C64)   # one source: no pencil
    n = ctypes.c_size_t(0)
    assert lib.dfm_initialise_workspace_size(ctypes.byref(one), ctypes.byref(n)) == 2
    fake = ctypes.c_void_p(0x1000)
    two = binding.make_problem(3, 10, (2, 2), 2, 2, binding.DFM_C64)
    assert lib.dfm_initialise(ctypes.byref(two), None, fake, fake, None, fake, 1 << 20, None) == 1
    assert lib.dfm_initialise(ctypes.byref(two), fake, fake, fake, None, fake, 16, None) == 3


def test_initialise_reports_a_singular_image_covariance():
    F, T, mics, N, K = 3, 40, (2, 2), 3, 2
    _, C = synth.source_images(F, T, mics, N, K, seed=1)
    C[-1, 1] = 0.0   # the last source silent in bin 1: R_f,N = 0
    with pytest.raises(binding.DFMError) as e:
        binding.initialise(C, mics)
    assert e.value.status == 6
