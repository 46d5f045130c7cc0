"""FP64 CPU oracle of distributed FastMNMF -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import anything under ``oracle/``.  The library product path never
does, and has no CPU fallback.

* ``oracle.dfmnmf``       -- the method itself: eqs. (2), (8)-(10), (13)-(16),
  the iteration schedule and the per-subarray multichannel Wiener filter.
* ``oracle.conventional`` -- conventional FastMNMF, eqs. (4)-(7) with (8)-(10),
  written separately in the paper's notation (pin for L = 1 and per-block IP).
* ``oracle.fullcov``      -- brute force from the full covariance of eq. (1) and
  the appendix theorem's commutator test.
* ``oracle.init``         -- the initial parameters from source-image estimates
  (Sec. IV-A, steps 3, 5 and 6), pinned by ``tests/test_oracle_init.py``.
* ``oracle.grad``         -- the cost after unrolled MM iterations written in PyTorch
  float64 and its gradient by torch.autograd, pinned by ``tests/test_oracle_grad.py``.

Every function is pinned by ``-m "not gpu"`` tests: ``tests/test_oracle_pins.py``
(brute force, closed forms, special cases, finite-difference identities,
monotonicity) and ``tests/test_oracle_floors.py`` (the 1e-6 floors of Sec. IV-A
with each floor active).  ``tests/test_oracle_mutations.py`` plants mistakes in a
copy of ``dfmnmf.py`` and checks that each one fails a pin.
"""
from . import conventional, dfmnmf, fullcov, grad, init  # noqa: F401
