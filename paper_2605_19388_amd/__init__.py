"""Distributed FastMNMF on AMD MI355X (gfx950).

The per-iteration hot path -- weighted covariances, iterative-projection
solves, |Qx|^2 and the multiplicative NMF / diagonal-SCM updates -- runs as
hand-written HIP kernels behind the C ABI declared in ``include/dfmnmf.h``
(shared library ``libdfmnmf.so`` in this package).  ``DistributedFastMNMF``
is a thin ctypes binding over that ABI; PyTorch only supplies device memory
and the HIP stream.

Importing the package does not load the library; touching the binding does,
and fails loudly if the library has not been built.
"""

__all__ = ["DistributedFastMNMF", "DFMError", "lib", "synth"]


def __getattr__(name):
    import importlib
    if name in ("DistributedFastMNMF", "DFMError", "lib"):
        return getattr(importlib.import_module(__name__ + ".binding"), name)
    if name in ("synth", "binding"):
        return importlib.import_module(__name__ + "." + name)
    raise AttributeError(name)
