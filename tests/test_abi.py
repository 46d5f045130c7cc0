"""The C-ABI library loads, exports every function include/dfmnmf.h declares, and
validates arguments on the host (CPU only: no call here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dfmnmf.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2605_19388_amd import binding, build
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    return binding.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dfm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("dfm_workspace_size", "dfm_init", "dfm_step", "dfm_nll", "dfm_separate", "dfm_destroy"):
        assert must in names


def test_library_exports_every_declared_function(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_function():
    from paper_2605_19388_amd import binding
    assert set(declared_functions()) <= set(binding.EXPORTS)


def _problem(**kw):
    from paper_2605_19388_amd import binding
    args = dict(F=5, T=7, mics=(2, 2), N=2, K=3, dtype=0, eps=1e-6, flags=0)
    args.update(kw)
    return binding.make_problem(args["F"], args["T"], args["mics"], args["N"], args["K"],
                                args["dtype"], args["eps"], args["flags"])


def _ws(lib, p):
    n = ctypes.c_size_t(0)
    return lib.dfm_workspace_size(ctypes.byref(p), ctypes.byref(n)), n.value


def test_workspace_size_valid(lib):
    st, n = _ws(lib, _problem())
    assert st == 0 and n > 0
    st64, n64 = _ws(lib, _problem(dtype=1))
    assert st64 == 0 and n64 > n


@pytest.mark.parametrize("kw,code", [
    (dict(F=0), 2), (dict(T=0), 2), (dict(N=0), 2), (dict(N=17), 2), (dict(K=0), 2), (dict(K=65), 2),
    (dict(mics=(2, 0)), 2), (dict(mics=(33,)), 2), (dict(mics=(32, 33)), 2), (dict(mics=(16,) * 5), 2),
    (dict(mics=()), 2), (dict(dtype=2), 1), (dict(eps=0.0), 1), (dict(eps=-1.0), 1), (dict(eps=float("nan")), 1),
    (dict(flags=16), 1), (dict(flags=1 << 31), 1),
    (dict(flags=4, mics=(2, 3)), 1),                      # BF16 covariances: generic partition
    (dict(flags=4, mics=(16,), N=5, K=16), 1),            # 16-mic blocks
    (dict(flags=4, mics=(4, 4, 4, 4), N=5, K=16, dtype=1), 1),  # complex128
])
def test_workspace_size_rejects(lib, kw, code):
    st, _ = _ws(lib, _problem(**kw))
    assert st == code


@pytest.mark.parametrize("kw", [dict(mics=(32,)), dict(mics=(32, 32)), dict(mics=(1,) * 64),
                                dict(flags=1), dict(flags=2), dict(flags=8), dict(flags=1 | 2 | 8),
                                dict(flags=4, mics=(4, 4, 4, 4), N=5, K=16), dict(flags=4, mics=(2, 2), N=2, K=4),
                                dict(flags=4, mics=(4, 4, 4), N=3, K=16)])
def test_workspace_size_accepts(lib, kw):
    st, n = _ws(lib, _problem(**kw))
    assert st == 0 and n > 0


def test_cost_trace_takes_workspace(lib):
    from paper_2605_19388_amd import binding
    _, plain = _ws(lib, _problem())
    _, traced = _ws(lib, _problem(flags=binding.F_TRACE_NLL))
    assert traced >= plain + 8 * binding.TRACE_CAPACITY


def test_separate_output_is_validated_before_any_launch():
    """A caller's output tensor of the wrong shape, dtype, device or layout is refused on the host
    (the Wiener-filter kernel writes N*F*T*M entries from its base pointer, unchecked)."""
    import torch
    from paper_2605_19388_amd import binding
    shape, dt, dev = (2, 3, 4, 5), torch.complex64, torch.device("cpu")
    binding.check_output(torch.empty(shape, dtype=dt), shape, dt, dev)
    bad = [torch.empty((2, 3, 4, 4), dtype=dt), torch.empty(shape, dtype=torch.complex128),
           torch.empty((2, 3, 5, 4), dtype=dt).transpose(2, 3), torch.empty(shape, dtype=dt, device="meta"),
           torch.empty(shape, dtype=dt).numpy()]
    for out in bad:
        with pytest.raises(binding.DFMError) as e:
            binding.check_output(out, shape, dt, dev)
        assert e.value.status == 1


def test_null_arguments_are_rejected(lib):
    p = _problem()
    assert lib.dfm_workspace_size(None, None) == 1
    n = ctypes.c_size_t(0)
    assert lib.dfm_workspace_size(None, ctypes.byref(n)) == 1
    plan = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    # missing buffers -> DFM_E_ARG before any device work
    assert lib.dfm_init(ctypes.byref(plan), ctypes.byref(p), None, fake, fake, fake, fake, fake, 1 << 30, None) == 1
    assert lib.dfm_init(None, ctypes.byref(p), fake, fake, fake, fake, fake, fake, 1 << 30, None) == 1
    # misaligned or short workspace -> DFM_E_WORKSPACE
    assert lib.dfm_init(ctypes.byref(plan), ctypes.byref(p), fake, fake, fake, fake, fake,
                        ctypes.c_void_p(0x1001), 1 << 30, None) == 3
    assert lib.dfm_init(ctypes.byref(plan), ctypes.byref(p), fake, fake, fake, fake, fake, fake, 16, None) == 3
    # bad shapes are found before pointers are used
    bad = _problem(N=0)
    assert lib.dfm_init(ctypes.byref(plan), ctypes.byref(bad), fake, fake, fake, fake, fake, fake, 1 << 30, None) == 2
    assert lib.dfm_step(None, 1, None) == 1
    assert lib.dfm_substep(None, 0, None) == 1
    out = ctypes.c_double()
    assert lib.dfm_nll(None, ctypes.byref(out), None) == 1
    cnt = ctypes.c_int32()
    assert lib.dfm_nll_trace(None, ctypes.byref(out), 1, ctypes.byref(cnt), None) == 1
    assert lib.dfm_separate(None, fake, None) == 1
    assert lib.dfm_covariances(None, fake, None) == 1
    assert lib.dfm_sync_status(None, None) == 1
    for kind in ("mm", "iter"):  # the gradients' entries
        assert getattr(lib, f"dfm_{kind}_tape_size")(None, 1, ctypes.byref(n)) == 1
        assert getattr(lib, f"dfm_{kind}_forward")(None, 1, fake, 1 << 20, None) == 1
        assert getattr(lib, f"dfm_{kind}_backward")(None, 1, fake, 1 << 20, fake, fake, fake, fake, None) == 1
    lib.dfm_destroy(None)


def test_gradient_tape_kind_is_checked_before_any_launch():
    """A tape recorded by the MM-only forward is refused by the full-iteration backward (and the
    other way round) in the binding, before the library is called."""
    import types
    import torch
    from paper_2605_19388_amd.binding import DistributedFastMNMF
    fake_plan = types.SimpleNamespace(_torch=torch)
    for kind, recorded in (("iter", "mm"), ("mm", "iter")):
        with pytest.raises(ValueError):
            DistributedFastMNMF._grad_backward(fake_plan, kind, (None, 0x1000, 1 << 20, 1, recorded))


def test_status_strings(lib):
    for code in range(7):
        s = lib.dfm_status_string(code)
        assert isinstance(s, bytes) and len(s) > 0
    assert lib.dfm_status_string(0) == b"ok"
