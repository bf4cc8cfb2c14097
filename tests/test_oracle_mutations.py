"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's filter-bank source (a
flipped sign, swapped operands, a dropped normalisation, a wrong exponent),
loads the copy as a module and runs every pin of tests/test_oracle_filterbank.py
against it: at least one pin must fail.  Everything here runs on the CPU.
"""
import importlib.util
import inspect
import os
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load(path, name):
    spec = importlib.util.spec_from_file_location(name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _mutant(old, new):
    path = os.path.join(ROOT, "oracle", "filterbank.py")
    src = open(path).read()
    assert src.count(old) >= 1, old
    mod = types.ModuleType("oracle.filterbank_mutant")
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new, 1), path, "exec"), mod.__dict__)
    return mod


def _calls(fn):
    """Argument sets of a (possibly parametrized) test function."""
    marks = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
    if not marks:
        return [{}]
    out = [{}]
    for m in marks:
        names = [n.strip() for n in m.args[0].split(",")] if isinstance(m.args[0], str) else list(m.args[0])
        nxt = []
        for base in out:
            for vals in m.args[1]:
                vals = vals if len(names) > 1 else (vals,)
                nxt.append({**base, **dict(zip(names, vals))})
        out = nxt
    return out


MUTATIONS = {
    "deviation sign flipped": ("- np.abs(es * ph_o - os_ * ph_e)", "+ np.abs(es * ph_o - os_ * ph_e)"),
    "phi_e / phi_o swapped in the deviation": ("np.abs(es * ph_o - os_ * ph_e)", "np.abs(es * ph_e - os_ * ph_o)"),
    "spread not normalised by N_s - 1": ("/ (p.n_scales - 1)", ""),
    "sigmoid centred the wrong way": ("p.g * (p.cutoff - spread)", "p.g * (spread - p.cutoff)"),
    "low-pass order halved": ("** (2 * p.lp_order)", "** (p.lp_order)"),
    "noise median on the largest scale": ("noise_threshold(np.abs(eo[0]), p)", "noise_threshold(np.abs(eo[-1]), p)"),
    "Rayleigh sigma factor dropped": ("math.sqrt((4.0 - math.pi) / 2.0)", "1.0"),
    "angular distance not wrapped": ("np.abs(np.arctan2(ds, dc))", "np.abs(theta - th_o)"),
    "radial log-Gaussian width squared twice": ("math.log(p.sigma_onf) ** 2", "math.log(p.sigma_onf) ** 4"),
    "moment b without its factor 2": ("b += 2.0 * pcc * pcs_", "b += pcc * pcs_"),
    "MIM ties to the highest orientation": ("upd = s_a > best", "upd = s_a >= best"),
    "Nyquist line left in the bank": ("g[nyq] = 0.0", "pass"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_a_planted_mistake_fails_a_pin(name):
    pins = _load(os.path.join(ROOT, "tests", "test_oracle_filterbank.py"), "pins_under_mutation")
    pins.fb = _mutant(*MUTATIONS[name])
    failed = []
    for fname, fn in inspect.getmembers(pins, inspect.isfunction):
        if not fname.startswith("test_") or fn.__module__ != pins.__name__:
            continue
        for kw in _calls(fn):
            try:
                fn(**kw)
            except AssertionError:
                failed.append(fname)
                break
            except Exception:  # noqa: BLE001 - a crash of the mutant also counts as caught
                failed.append(fname)
                break
    assert failed, f"no pin fails with the mistake: {name}"
