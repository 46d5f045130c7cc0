"""ctypes binding of the C ABI in ``include/dfmnmf.h``.

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libdfmnmf.so``.  PyTorch provides device memory (the state tensors and
the workspace) and the current HIP stream.  There is no CPU fallback: if the
library is missing or no GPU is present, constructing a plan raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdfmnmf.so")

MAX_SUBARRAYS = 64
DFM_C64, DFM_C128 = 0, 1
# dfm_problem.flags bits
F_CHECK_FINITE, F_TRACE_NLL, F_GRAM_BF16, F_NO_GRAPH = 1, 2, 4, 8
TRACE_CAPACITY = 4096
NOALLOC_SCRATCH_BYTES = 64 << 20
STAGES = {"ip": 0, "W": 1, "H": 2, "g": 3}
STATUS = {0: "DFM_OK", 1: "DFM_E_ARG", 2: "DFM_E_SHAPE", 3: "DFM_E_WORKSPACE", 4: "DFM_E_HIP",
          5: "DFM_E_NONFINITE", 6: "DFM_E_SINGULAR"}


class DFMError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = int(status)
        msg = STATUS.get(self.status, f"status {status}")
        if _lib is not None:
            msg += ": " + _lib.dfm_status_string(self.status).decode()
        super().__init__(f"{where}: {msg}" if where else msg)


class Problem(ctypes.Structure):
    _fields_ = [("F", ctypes.c_int32), ("T", ctypes.c_int32), ("N", ctypes.c_int32),
                ("K", ctypes.c_int32), ("L", ctypes.c_int32),
                ("mics", ctypes.c_int32 * MAX_SUBARRAYS), ("dtype", ctypes.c_int32),
                ("eps", ctypes.c_double), ("flags", ctypes.c_uint32), ("tile", ctypes.c_int32)]


_lib = None
EXPORTS = ("dfm_workspace_size", "dfm_init", "dfm_step", "dfm_substep", "dfm_nll", "dfm_nll_trace", "dfm_separate",
           "dfm_covariances", "dfm_sync_status", "dfm_kernel_times", "dfm_profile_kernel", "dfm_profile_read",
           "dfm_kernel_count", "dfm_kernel_name", "dfm_run_noalloc", "dfm_initialise_workspace_size",
           "dfm_initialise", "dfm_mm_tape_size", "dfm_mm_forward", "dfm_mm_backward", "dfm_iter_tape_size",
           "dfm_iter_forward", "dfm_iter_backward", "dfm_batch_create",
           "dfm_batch_step", "dfm_batch_destroy", "dfm_destroy", "dfm_status_string")


def load(path: str = LIB_PATH):
    """Load libdfmnmf.so and declare its signatures.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise DFMError(4, f"{path} is missing; build it with `python -m paper_2605_19388_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
    P = ctypes.POINTER(Problem)
    lib.dfm_workspace_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.dfm_init.argtypes = [ctypes.POINTER(vp), P, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.dfm_step.argtypes = [vp, i32, vp]
    lib.dfm_substep.argtypes = [vp, i32, vp]
    lib.dfm_nll.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.dfm_nll_trace.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32), vp]
    lib.dfm_separate.argtypes = [vp, vp, vp]
    lib.dfm_covariances.argtypes = [vp, vp, vp]
    lib.dfm_sync_status.argtypes = [vp, vp]
    lib.dfm_kernel_times.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), vp]
    lib.dfm_profile_kernel.argtypes = [vp, i32, i32]
    lib.dfm_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), vp]
    lib.dfm_run_noalloc.argtypes = [P, vp, vp, vp, vp, vp, i32, vp, vp, vp]
    lib.dfm_initialise_workspace_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.dfm_initialise.argtypes = [P, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.dfm_mm_tape_size.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.dfm_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), i32]
    lib.dfm_batch_step.argtypes = [vp, i32, vp]
    lib.dfm_batch_destroy.argtypes = [vp]
    lib.dfm_batch_destroy.restype = None
    lib.dfm_mm_forward.argtypes = [vp, i32, vp, ctypes.c_size_t, vp]
    lib.dfm_mm_backward.argtypes = [vp, i32, vp, ctypes.c_size_t, vp, vp, vp, vp, vp]
    lib.dfm_iter_tape_size.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.dfm_iter_forward.argtypes = [vp, i32, vp, ctypes.c_size_t, vp]
    lib.dfm_iter_backward.argtypes = [vp, i32, vp, ctypes.c_size_t, vp, vp, vp, vp, vp]
    lib.dfm_kernel_count.argtypes = [vp]
    lib.dfm_kernel_count.restype = i32
    lib.dfm_kernel_name.argtypes = [vp, i32]
    lib.dfm_kernel_name.restype = ctypes.c_char_p
    lib.dfm_destroy.argtypes = [vp]
    lib.dfm_destroy.restype = None
    lib.dfm_status_string.argtypes = [st]
    lib.dfm_status_string.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("dfm_kernel_count", "dfm_kernel_name", "dfm_destroy", "dfm_batch_destroy", "dfm_status_string"):
            getattr(lib, name).restype = st
    _lib = lib
    return lib


def lib():
    return load()


def make_problem(F, T, mics, N, K, dtype=DFM_C64, eps=1e-6, flags=0, tile=0) -> Problem:
    p = Problem()
    p.F, p.T, p.N, p.K, p.L = int(F), int(T), int(N), int(K), len(mics)
    if len(mics) > MAX_SUBARRAYS:
        raise DFMError(2, "too many subarrays")
    for i, m in enumerate(mics):
        p.mics[i] = int(m)
    p.dtype = int(dtype)
    p.eps = float(eps)
    p.flags = int(flags)
    p.tile = int(tile)
    return p


def workspace_size(problem: Problem) -> int:
    n = ctypes.c_size_t(0)
    st = load().dfm_workspace_size(ctypes.byref(problem), ctypes.byref(n))
    if st:
        raise DFMError(st, "dfm_workspace_size")
    return int(n.value)


def _check(st, where):
    if st:
        raise DFMError(st, where)


def check_output(out, shape, dtype, device):
    """A caller-supplied output tensor must be exactly what the kernel writes: the kernels
    store every element of `shape` from out.data_ptr() on, with no bounds of their own."""
    import torch
    if not isinstance(out, torch.Tensor):
        raise DFMError(1, "out must be a torch tensor")
    if tuple(out.shape) != tuple(shape):
        raise DFMError(1, f"out has shape {tuple(out.shape)}, expected {tuple(shape)}")
    if out.dtype != dtype:
        raise DFMError(1, f"out has dtype {out.dtype}, expected {dtype}")
    if out.device != torch.device(device):
        raise DFMError(1, f"out is on {out.device}, expected {device}")
    if not out.is_contiguous():
        raise DFMError(1, "out must be contiguous")


class Batch:
    """Steps several DistributedFastMNMF plans together (dfm_batch_*): one graph launch per phase
    runs every plan's kernels, each plan a branch of the graph.  Each plan's result equals its own
    step(n) bit for bit.  Keeps references to the plans."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._plan.value for p in self.plans])
        self._b = ctypes.c_void_p()
        _check(load().dfm_batch_create(ctypes.byref(self._b), arr, len(self.plans)), "dfm_batch_create")

    def step(self, n_iter: int = 1):
        _check(load().dfm_batch_step(self._b, int(n_iter), self.plans[0]._stream()), "dfm_batch_step")
        return self

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            load().dfm_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def initialise(C, mics, with_h=True, device="cuda"):
    """Initial Q, g (and h) from source-image estimates C [N, F, T, M] (complex64 or complex128;
    numpy array or torch tensor), by dfm_initialise (Sec. IV-A, steps 3, 5, 6).  Returns torch
    tensors on `device`: Q [F, sum M_l^2], g [F, N, M], h [N, F, T] (None unless with_h)."""
    import torch
    lib_ = load()
    if not torch.cuda.is_available():
        raise DFMError(4, "no GPU visible to HIP")
    dev = torch.device(device)
    Ct = torch.as_tensor(C)
    if Ct.dtype not in (torch.complex64, torch.complex128):
        raise DFMError(1, "C must be complex64 or complex128")
    Ct = Ct.to(dev).contiguous()
    N, F, T, M = Ct.shape
    mics = tuple(int(m) for m in mics)
    if sum(mics) != M:
        raise DFMError(2, "sum(mics) != C.shape[3]")
    dtype = DFM_C64 if Ct.dtype == torch.complex64 else DFM_C128
    rdt = torch.float32 if dtype == DFM_C64 else torch.float64
    prob = make_problem(F, T, mics, N, 1, dtype)
    n = ctypes.c_size_t(0)
    _check(lib_.dfm_initialise_workspace_size(ctypes.byref(prob), ctypes.byref(n)), "dfm_initialise_workspace_size")
    ws = torch.empty(n.value + 256, dtype=torch.uint8, device=dev)
    ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
    Q = torch.empty((F, sum(m * m for m in mics)), dtype=Ct.dtype, device=dev)
    g = torch.empty((F, N, M), dtype=rdt, device=dev)
    h = torch.empty((N, F, T), dtype=rdt, device=dev) if with_h else None
    st = lib_.dfm_initialise(ctypes.byref(prob), Ct.data_ptr(), Q.data_ptr(), g.data_ptr(),
                             h.data_ptr() if with_h else None, ptr, n.value,
                             torch.cuda.current_stream(dev).cuda_stream)
    _check(st, "dfm_initialise")
    return Q, g, h


class DistributedFastMNMF:
    """Distributed FastMNMF plan on one GPU.

    X: [F, T, M] complex (numpy array or torch tensor); complex64 runs the FP32
    path, complex128 the FP64 path.  mics: subarray sizes (contiguous columns of X).
    W [N, F, K] and H [N, K, T] are required (the library draws no random numbers);
    Q defaults to the block identity and g to ones.  All state lives in device
    tensors owned by this object and is updated in place by ``step``.
    """

    def __init__(self, X, mics, n_src, n_basis, W, H, Q=None, g=None, eps=1e-6, device="cuda", flags=0, tile=0):
        import torch

        self._torch = torch
        lib_ = load()
        if not torch.cuda.is_available():
            raise DFMError(4, "no GPU visible to HIP")
        dev = torch.device(device)
        Xt = torch.as_tensor(X)
        if Xt.dtype not in (torch.complex64, torch.complex128):
            raise DFMError(1, "X must be complex64 or complex128")
        self.dtype = DFM_C64 if Xt.dtype == torch.complex64 else DFM_C128
        cdt = Xt.dtype
        rdt = torch.float32 if self.dtype == DFM_C64 else torch.float64
        F, T, M = Xt.shape
        self.mics = tuple(int(m) for m in mics)
        if sum(self.mics) != M:
            raise DFMError(2, "sum(mics) != X.shape[2]")
        self.F, self.T, self.M, self.N, self.K = int(F), int(T), int(M), int(n_src), int(n_basis)
        self.X = Xt.to(dev).contiguous()
        qf = sum(m * m for m in self.mics)
        if Q is None:
            Q = np.zeros((F, qf), dtype=np.complex128)
            o = 0
            for m in self.mics:
                Q[:, o:o + m * m] = np.eye(m).ravel()
                o += m * m
        if g is None:
            g = np.ones((F, self.N, M))
        self.Q = torch.as_tensor(Q).to(device=dev, dtype=cdt).contiguous().clone()
        self.g = torch.as_tensor(g).to(device=dev, dtype=rdt).contiguous().clone()
        self.W = torch.as_tensor(W).to(device=dev, dtype=rdt).contiguous().clone()
        self.H = torch.as_tensor(H).to(device=dev, dtype=rdt).contiguous().clone()
        for name, t, shp in (("Q", self.Q, (F, qf)), ("g", self.g, (F, self.N, M)),
                             ("W", self.W, (self.N, F, self.K)), ("H", self.H, (self.N, self.K, T))):
            if tuple(t.shape) != shp:
                raise DFMError(2, f"{name} has shape {tuple(t.shape)}, expected {shp}")
        self.problem = make_problem(F, T, self.mics, self.N, self.K, self.dtype, eps, flags, tile)
        nbytes = workspace_size(self.problem)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-self._ws.data_ptr()) % 256
        self._ws_ptr = self._ws.data_ptr() + off
        self._ws_bytes = nbytes
        self.device = self.X.device  # with its index (cuda:0), for comparisons
        self._plan = ctypes.c_void_p()
        st = lib_.dfm_init(ctypes.byref(self._plan), ctypes.byref(self.problem),
                           self.X.data_ptr(), self.Q.data_ptr(), self.g.data_ptr(), self.W.data_ptr(),
                           self.H.data_ptr(), self._ws_ptr, self._ws_bytes, self._stream())
        _check(st, "dfm_init")

    def _stream(self):
        return self._torch.cuda.current_stream(self.device).cuda_stream

    def step(self, n_iter: int = 1):
        _check(load().dfm_step(self._plan, int(n_iter), self._stream()), "dfm_step")
        return self

    def substep(self, stage):
        stage = STAGES[stage] if isinstance(stage, str) else int(stage)
        _check(load().dfm_substep(self._plan, stage, self._stream()), "dfm_substep")
        return self

    def nll(self) -> float:
        out = ctypes.c_double(0.0)
        _check(load().dfm_nll(self._plan, ctypes.byref(out), self._stream()), "dfm_nll")
        return float(out.value)

    def nll_trace(self):
        """Costs (13) recorded after each iteration of step() (plan made with F_TRACE_NLL)."""
        buf = (ctypes.c_double * TRACE_CAPACITY)()
        n = ctypes.c_int32(0)
        _check(load().dfm_nll_trace(self._plan, buf, TRACE_CAPACITY, ctypes.byref(n), self._stream()),
               "dfm_nll_trace")
        return np.array(buf[:min(n.value, TRACE_CAPACITY)]), int(n.value)

    def separate(self, out=None):
        torch = self._torch
        shape = (self.N, self.F, self.T, self.M)
        if out is None:
            out = torch.empty(shape, dtype=self.X.dtype, device=self.device)
        else:
            check_output(out, shape, self.X.dtype, self.device)
        _check(load().dfm_separate(self._plan, out.data_ptr(), self._stream()), "dfm_separate")
        return out

    def covariances(self):
        torch = self._torch
        vc = sum(m ** 3 for m in self.mics)
        out = torch.empty((self.F, vc), dtype=self.X.dtype, device=self.device)
        _check(load().dfm_covariances(self._plan, out.data_ptr(), self._stream()), "dfm_covariances")
        return out

    def kernel_names(self):
        lib_ = load()
        return [lib_.dfm_kernel_name(self._plan, i).decode() for i in range(lib_.dfm_kernel_count(self._plan))]

    def kernel_times(self, reps: int = 20):
        """Average ms per launch of every kernel of one iteration (changes the state)."""
        lib_ = load()
        n = lib_.dfm_kernel_count(self._plan)
        out = (ctypes.c_double * n)()
        _check(lib_.dfm_kernel_times(self._plan, int(reps), out, self._stream()), "dfm_kernel_times")
        return dict(zip(self.kernel_names(), list(out)))

    def profile_kernel(self, name_or_index, max_launches: int = 4096):
        k = -1 if name_or_index is None else (
            self.kernel_names().index(name_or_index) if isinstance(name_or_index, str) else int(name_or_index))
        _check(load().dfm_profile_kernel(self._plan, k, int(max_launches)), "dfm_profile_kernel")

    def profile_read(self):
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        _check(load().dfm_profile_read(self._plan, ctypes.byref(ms), ctypes.byref(n), self._stream()),
               "dfm_profile_read")
        return float(ms.value), int(n.value)

    def sync_status(self):
        _check(load().dfm_sync_status(self._plan, self._stream()), "dfm_sync_status")

    def _grad_forward(self, kind: str, n_iter: int):
        torch = self._torch
        lib_ = load()
        n = ctypes.c_size_t(0)
        _check(getattr(lib_, f"dfm_{kind}_tape_size")(self._plan, int(n_iter), ctypes.byref(n)),
               f"dfm_{kind}_tape_size")
        buf = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        ptr = buf.data_ptr() + (-buf.data_ptr()) % 256
        _check(getattr(lib_, f"dfm_{kind}_forward")(self._plan, int(n_iter), ptr, n.value, self._stream()),
               f"dfm_{kind}_forward")
        return (buf, ptr, n.value, int(n_iter), kind)

    def _grad_backward(self, kind: str, tape):
        torch = self._torch
        _, ptr, nbytes, n_iter, recorded = tape
        if recorded != kind:
            raise ValueError(f"tape recorded by {recorded}_forward, not {kind}_forward")
        dQ, dg, dW, dH = (torch.empty_like(t) for t in (self.Q, self.g, self.W, self.H))
        _check(getattr(load(), f"dfm_{kind}_backward")(self._plan, n_iter, ptr, nbytes, dQ.data_ptr(), dg.data_ptr(),
                                                        dW.data_ptr(), dH.data_ptr(), self._stream()),
               f"dfm_{kind}_backward")
        return dQ, dg, dW, dH

    def mm_forward(self, n_iter: int):
        """n_iter MM iterations (8)-(10) with Q fixed, recording per-iteration checkpoints; returns
        the tape to pass to mm_backward."""
        return self._grad_forward("mm", n_iter)

    def mm_backward(self, tape):
        """Gradient of the cost after the recorded MM iterations with respect to the state before
        them: (dQ, dg, dW, dH) device tensors (dQ = dL/dRe Q + i dL/dIm Q)."""
        return self._grad_backward("mm", tape)

    def iter_forward(self, n_iter: int):
        """n_iter full iterations (eq. (14), the IP sweep (15)-(16), then (8)-(10)), recording
        per-iteration checkpoints of (Q, g, W, H); returns the tape to pass to iter_backward."""
        return self._grad_forward("iter", n_iter)

    def iter_backward(self, tape):
        """Gradient of the cost after the recorded full iterations with respect to the state before
        them: (dQ, dg, dW, dH) device tensors (dQ = dL/dRe Q + i dL/dIm Q)."""
        return self._grad_backward("iter", tape)

    def load_state(self, Q=None, g=None, W=None, H=None):
        """Copy new values into the state tensors in place (the plan keeps their addresses)."""
        torch = self._torch
        for name, v in (("Q", Q), ("g", g), ("W", W), ("H", H)):
            if v is not None:
                t = getattr(self, name)
                t.copy_(torch.as_tensor(v).to(device=self.device, dtype=t.dtype).reshape(t.shape))
        return self

    def state(self):
        """Host copies (numpy) of Q, g, W, H."""
        self._torch.cuda.synchronize(self.device)
        return {k: getattr(self, k).cpu().numpy() for k in ("Q", "g", "W", "H")}

    def close(self):
        if getattr(self, "_plan", None) and self._plan.value:
            load().dfm_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
