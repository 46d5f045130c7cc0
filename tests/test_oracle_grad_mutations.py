"""The gradient oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of ``oracle/grad.py`` (built from the source text in
memory; nothing on disk changes) and runs every test of tests/test_oracle_grad.py against the copy:
at least one must fail, and the unmodified module must pass them all.  The mistakes cover the
forward (eq. (14), the sweep of eqs. (15)-(16), the iteration order, the cost (13)) and paths of
the gradient cut while the forward value stays the same (a detached weight or normaliser), which
only the finite-difference pins can see.
"""
import inspect
import itertools
import os
import types

import pytest

import tests.test_oracle_grad as pins

GRAD_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "grad.py")

# name -> list of (text in the module, replacement).
MUTANTS = {
    "cov_conj_dropped": [('"ftu,fta,ftb->fuab", w, xl, xl.conj()', '"ftu,fta,ftb->fuab", w, xl, xl')],
    "cov_1_over_T_dropped": [('w, xl, xl.conj()) / T)', 'w, xl, xl.conj()))')],
    "cov_weight_not_inverted": [("w = (1.0 / y[:, :, mo:mo + ml])", "w = (y[:, :, mo:mo + ml])")],
    "cov_weight_detached": [("w = (1.0 / y[:, :, mo:mo + ml]).to(X.dtype)",
                             "w = (1.0 / y[:, :, mo:mo + ml]).detach().to(X.dtype)")],
    "sweep_rows_descending": [("for mu in range(ml):\n            e = ", "for mu in reversed(range(ml)):\n            e = ")],
    "sweep_operands_swapped": [("torch.linalg.solve(Ql @ Vl[:, mu], e)", "torch.linalg.solve(Vl[:, mu] @ Ql, e)")],
    "sweep_row_unconjugated": [("b.conj()[:, None, :]", "b[:, None, :]")],
    "sweep_normaliser_sqrt_dropped": [("b / torch.sqrt(torch.clamp(s, min=eps))", "b / torch.clamp(s, min=eps)")],
    "sweep_normaliser_floor_removed": [("b / torch.sqrt(torch.clamp(s, min=eps))", "b / torch.sqrt(s)")],
    "sweep_normaliser_floor_1e-3": [("b / torch.sqrt(torch.clamp(s, min=eps))", "b / torch.sqrt(torch.clamp(s, min=1e-3))")],
    "y_floor_removed": [("return lam, torch.clamp(torch.einsum(\"ftn,fnm->ftm\", lam, g), min=eps)",
                         "return lam, torch.einsum(\"ftn,fnm->ftm\", lam, g)")],
    "sweep_normaliser_detached": [("b / torch.sqrt(torch.clamp(s, min=eps))",
                                   "b / torch.sqrt(torch.clamp(s.detach(), min=eps))")],
    "powers_from_the_old_Q": [("        Q = ip_sweep(Q, covariances", "        Qn = ip_sweep(Q, covariances"),
                              ("        P = powers(X, Q, mics)\n        W = update_W(W, H, g, P, eps)\n        H = update_H(W, H, g, P, eps)\n        g = update_g(W, H, g, P, eps)\n    return cost(X, Q, g, W, H, mics, eps)",
                               "        P = powers(X, Q, mics)\n        Q = Qn\n        W = update_W(W, H, g, P, eps)\n        H = update_H(W, H, g, P, eps)\n        g = update_g(W, H, g, P, eps)\n    return cost(X, Q, g, W, H, mics, eps)")],
    "sweep_before_the_model_of_the_state": [("        _, y = model(W, H, g, eps)\n        Q = ip_sweep(",
                                             "        _, y = model(W * 1.01, H, g, eps)\n        Q = ip_sweep(")],
    "cost_logdet_factor_T": [("- 2.0 * T * logdet", "- T * logdet")],
    "W_update_y_not_squared": [("num = torch.einsum(\"nkt,fnm,ftm->nfk\", H, g, P / y ** 2)",
                                "num = torch.einsum(\"nkt,fnm,ftm->nfk\", H, g, P / y)")],
    "g_update_denominator_floor_detached": [("return g * torch.sqrt(num / torch.clamp(den, min=eps))",
                                             "return g * torch.sqrt(num / torch.clamp(den, min=eps).detach())")],
}


def _mutant(name):
    src = open(GRAD_SRC).read().replace("from .dfmnmf import", "from oracle.dfmnmf import")
    for old, new in MUTANTS[name]:
        assert src.count(old) == 1, f"{name}: {old!r} occurs {src.count(old)} times in the module"
        src = src.replace(old, new)
    mod = types.ModuleType(f"grad_mutant_{name}")
    exec(compile(src, f"<mutant {name}>", "exec"), mod.__dict__)
    return mod


def _pin_calls():
    """Every test of test_oracle_grad, expanded over its parametrisations."""
    calls = []
    for fname, fn in inspect.getmembers(pins, inspect.isfunction):
        if not fname.startswith("test_"):
            continue
        marks = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
        grids = []
        for m in marks:
            argnames = m.args[0]
            argnames = [a.strip() for a in argnames.split(",")] if isinstance(argnames, str) else list(argnames)
            grids.append([(argnames, v if len(argnames) > 1 else (v,)) for v in m.args[1]])
        for combo in itertools.product(*grids):
            kw = {}
            for argnames, vals in combo:
                kw.update(dict(zip(argnames, vals)))
            calls.append((f"{fname}{kw}", fn, kw))
    return calls


def _run(module):
    """Names of the pins that fail with `module` as the gradient oracle."""
    failed = []
    saved = pins.G
    pins.G = module
    try:
        for name, fn, kw in CALLS:
            try:
                fn(**kw)
            except Exception:  # an AssertionError, or the mistake breaking the computation outright
                failed.append(name)
    finally:
        pins.G = saved
    return failed


CALLS = _pin_calls()


def test_unmodified_module_passes_every_pin():
    from oracle import grad
    assert _run(grad) == []


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(name):
    failed = _run(_mutant(name))
    assert failed, f"no pin fails with the mistake {name!r} planted in the gradient oracle"
