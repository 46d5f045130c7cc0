"""The oracle's pins catch plausible mistakes (CPU only).

Each case below plants one mistake in a copy of ``oracle/dfmnmf.py`` (the copy is
built from the source text in memory; nothing on disk changes), then runs every
pin of tests/test_oracle_pins.py and every floor check of
tests/test_oracle_floors.py against the copy.  The planted mistake must make at
least one of them fail, and the unmodified oracle must pass them all.  The
mistakes cover the floors of Sec. IV-A (removed, or at the wrong value), and a
dropped or wrong term, sign, index, operand order, exponent or loop order in
eqs. (2), (8)-(10) and (13)-(16), the iteration order and the Wiener filter.
"""
import inspect
import itertools
import os
import types

import pytest

import tests.test_oracle_floors as floors
import tests.test_oracle_pins as pins

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "dfmnmf.py")

# name -> list of (text in the oracle, replacement, occurrence to replace (0 = first)).
MUTANTS = {
    # floors (Sec. IV-A)
    "y_floor_removed": [("return np.maximum(y, eps)", "return y", 0)],
    "y_floor_1e-3": [("return np.maximum(y, eps)", "return np.maximum(y, 1e-3)", 0)],
    "mm_den_floor_removed": [("np.sqrt(num / np.maximum(den, eps))", "np.sqrt(num / den)", 0)],
    "mm_den_floor_1e-3": [("np.sqrt(num / np.maximum(den, eps))", "np.sqrt(num / np.maximum(den, 1e-3))", 0)],
    "normaliser_floor_removed": [("np.sqrt(np.maximum(s, eps))", "np.sqrt(s)", 0)],
    "normaliser_floor_1e-3": [("np.sqrt(np.maximum(s, eps))", "np.sqrt(np.maximum(s, 1e-3))", 0)],
    "default_floor_1e-4": [("EPS = 1e-6", "EPS = 1e-4", 0)],
    # eq. (2) / model
    "model_wrong_source_axis": [('np.einsum("ftn,fnm->ftm", lam, g, optimize=True)',
                                 'np.einsum("ftn,fnm->ftm", lam[:, :, ::-1], g, optimize=True)', 0)],
    # eq. (14)
    "gram_conj_dropped": [("w, xl, xl.conj()", "w, xl, xl", 0)],
    "gram_conj_on_wrong_side": [("w, xl, xl.conj()", "w, xl.conj(), xl", 0)],
    "gram_1_over_T_dropped": [("optimize=True) / T)", "optimize=True))", 0)],
    "gram_weight_of_wrong_mic": [("w = 1.0 / y[:, :, mo:mo + ml]", "w = 1.0 / y[:, :, :ml]", 0)],
    "gram_weight_not_inverted": [("w = 1.0 / y[:, :, mo:mo + ml]", "w = y[:, :, mo:mo + ml]", 0)],
    # eqs. (15)-(16)
    "ip_operands_swapped": [("A = Ql @ Vmu", "A = Vmu @ Ql", 0)],
    "ip_normaliser_sqrt_dropped": [("np.sqrt(np.maximum(s, eps))", "np.maximum(s, eps)", 0)],
    "ip_row_stored_unconjugated": [("out[:, mu, :] = w.conj()", "out[:, mu, :] = w", 0)],
    "ip_rows_descending": [("for mu in range(ml):\n            blocks[l]",
                            "for mu in reversed(range(ml)):\n            blocks[l]", 0)],
    "ip_normaliser_imag_part": [("einsum(\"fa,fab,fb->f\", w.conj(), Vmu, w).real",
                                 "einsum(\"fa,fab,fb->f\", w.conj(), Vmu, w).imag + 1.0", 0)],
    # powers |Q x|^2
    "powers_Q_transposed": [('np.einsum("fua,fta->ftu", Ql, X[:, :, mo:mo + ml], optimize=True)\n        P',
                             'np.einsum("fau,fta->ftu", Ql, X[:, :, mo:mo + ml], optimize=True)\n        P', 0)],
    # eqs. (8)-(10)
    "mm_exponent_one": [("return x * np.sqrt(num / np.maximum(den, eps))",
                         "return x * (num / np.maximum(den, eps))", 0)],
    "W_numerator_y_not_squared": [("P / y ** 2", "P / y", 0)],
    "H_denominator_uses_numerator_weights": [('den = np.einsum("nfk,ftn->nkt", W, b',
                                              'den = np.einsum("nfk,ftn->nkt", W, a', 0)],
    "H_sum_over_wrong_axis": [('num = np.einsum("nfk,ftn->nkt", W, a', 'num = np.einsum("nfk,ftn->nkt", W[:, ::-1], a', 0)],
    "g_denominator_y_squared": [('"ftn,ftm->fnm", lam, 1.0 / y,', '"ftn,ftm->fnm", lam, 1.0 / y ** 2,', 0)],
    "g_numerator_missing_lambda": [('"ftn,ftm->fnm", lam, P / y ** 2', '"ftn,ftm->fnm", lam ** 0, P / y ** 2', 0)],
    # iteration order (Sec. III-B)
    "powers_from_the_old_Q": [("        Q = ip_sweep(Q,", "        Q_old = Q\n        Q = ip_sweep(Q,", 0),
                              ("        P = powers(X, Q, mics)", "        P = powers(X, Q_old, mics)", 0)],
    "H_update_with_the_old_W": [("        W = update_W(W, H, g, P, eps)", "        W_old = W\n        W = update_W(W, H, g, P, eps)", 0),
                                ("        H = update_H(W, H, g, P, eps)", "        H = update_H(W_old, H, g, P, eps)", 0)],
    # eq. (13)
    "nll_logdet_factor_T": [("- 2.0 * T * np.sum(logabsdet", "- T * np.sum(logabsdet", 0)],
    "nll_log_sign": [("np.sum(P / y + np.log(y))", "np.sum(P / y - np.log(y))", 0)],
    "nll_unfloored_y_in_log": [("np.sum(P / y + np.log(y))",
                                "np.sum(P / y + np.log(np.einsum('ftn,fnm->ftm', source_psd(W, H), g)))", 0)],
    # Wiener filter
    "separate_inverse_transposed": [("Qinv = np.linalg.inv(Ql)", "Qinv = np.linalg.inv(Ql).T", 0)],
    "separate_gain_not_divided_by_y": [("/ y[:, :, mo:mo + ml]\n            S[",
                                        "/ y[:, :, mo:mo + ml] ** 0\n            S[", 0)],
}


def _mutant(name):
    src = open(ORACLE_SRC).read()
    for old, new, occ in MUTANTS[name]:
        count = src.count(old)
        assert count > occ, f"{name}: {old!r} occurs {count} times in the oracle"
        head, *rest = src.split(old)
        src = old.join([head] + rest[:occ]) + new + old.join(rest[occ:])
    mod = types.ModuleType(f"oracle_mutant_{name}")
    exec(compile(src, f"<mutant {name}>", "exec"), mod.__dict__)
    return mod


def _pin_calls():
    """Every pin of test_oracle_pins (expanded over its parametrisations) and every floor check."""
    calls = []
    for fname, fn in inspect.getmembers(pins, inspect.isfunction):
        if not fname.startswith("test_"):
            continue
        marks = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
        if not marks:
            calls.append((fname, fn, {}))
            continue
        names, grids = [], []
        for m in marks:
            argnames = m.args[0]
            argnames = [a.strip() for a in argnames.split(",")] if isinstance(argnames, str) else list(argnames)
            names.append(argnames)
            grids.append(list(m.args[1]))
        for combo in itertools.product(*grids):
            kw = {}
            for argnames, vals in zip(names, combo):
                vals = vals if len(argnames) > 1 else (vals,)
                kw.update(dict(zip(argnames, vals)))
            calls.append((f"{fname}{kw}", fn, kw))
    for cname, check in sorted(floors.FLOOR_CHECKS.items()):
        calls.append((f"floor:{cname}", None, {"check": check}))
    return calls


def _run(calls, module):
    """Names of the pins that fail with `module` as the oracle."""
    failed = []
    saved = pins.D, floors.D
    pins.D = floors.D = module
    try:
        for name, fn, kw in calls:
            try:
                if fn is None:
                    kw["check"](module)
                else:
                    fn(**kw)
            except Exception:  # an AssertionError, or the mistake breaking the computation outright
                failed.append(name)
    finally:
        pins.D, floors.D = saved
    return failed


CALLS = _pin_calls()


def test_unmodified_oracle_passes_every_pin():
    from oracle import dfmnmf
    assert _run(CALLS, dfmnmf) == []


@pytest.mark.filterwarnings("ignore::RuntimeWarning")  # some mistakes take square roots of negatives
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(name):
    failed = _run(CALLS, _mutant(name))
    assert failed, f"no pin fails with the mistake {name!r} planted in the oracle"
