"""The oracle's composed quantities against independent values
(tests/oracle_composition_pins.py), and planted mistakes in the Python layer
of the oracle (on the CPU) that those pins must catch."""
import importlib.util
import os
import shutil
import tempfile

import pytest

import oracle
from tests import oracle_composition_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "__init__.py")


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda c: c.__name__)
def test_composition_pin(check):
    check(oracle)


def test_every_composition_is_pinned():
    names = {c.__name__ for c in pins.ALL_CHECKS}
    for fn in ("weighted_sum", "backward", "backward_ld", "central_difference", "pairsum"):
        assert callable(getattr(oracle, fn))
        assert pins.PINS.get(fn), f"oracle.{fn} has no pin"
        assert set(pins.PINS[fn]) <= names


# Plausible mistakes in oracle/__init__.py: (text to find, replacement).
MUTANTS = {
    "ws_weight_offset_shifted": ("wl = w[wo:wo + k + 1]", "wl = w[wo + 1:wo + k + 2]"),
    "ws_k_weights_not_k_plus_1": ("wl = w[wo:wo + k + 1].astype(np.longdouble)",
                                  "wl = np.append(w[wo:wo + k], 0.0).astype(np.longdouble)"),
    "ws_orders_shifted": ("F = boys_ld(x[off:off + n], k, threads)",
                          "F = boys_ld(x[off:off + n], k + 1, threads)[:, 1:]"),
    "ws_output_not_cleared": ("out = np.zeros(x.size, dtype=np.float64)",
                              "out = np.array(x, dtype=np.float64)"),
    "ws_rows_shifted": ("out[off:off + n] = (F", "out[off + 1:off + n + 1] = (F"),
    "bw_wrong_columns": ("* F[:, 1:]).sum(axis=1)", "* F[:, :-1]).sum(axis=1)"),
    "bw_sign_dropped": ("return -(G.astype(np.longdouble)", "return (G.astype(np.longdouble)"),
    "cd_half_step": ("return ((Lp - Lm) / (2 * h))", "return ((Lp - Lm) / h)"),
    "cd_step_zero_at_origin": ("h = np.longdouble(rel_step) * np.maximum(np.longdouble(1), xl)",
                               "h = np.longdouble(rel_step) * xl"),
    "cd_one_sided": ("Fm = boys_ld(xl - h, K, threads)", "Fm = boys_ld(xl, K, threads)"),
    "ps_product_argument": ("F = boys_ld(x[int(i)] + x, k, threads)",
                            "F = boys_ld(x[int(i)] * x, k, threads)"),
    "ps_weights_reversed": ("w = (F * c[None, :]).sum(axis=1)", "w = (F * c[::-1][None, :]).sum(axis=1)"),
    "ps_y_dropped": ("z.append((y * w).sum())", "z.append(w.sum())"),
    "ps_rows_ignored": ("rows = range(x.size) if rows is None else rows",
                        "rows = range(x.size) if rows is None else range(len(rows))"),
}


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="oracle_py_mutants_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def _load_mutant(name, workdir):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = os.path.join(workdir, f"oracle_{name}.py")
    with open(path, "w") as f:
        f.write(text.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"oracle_{name}", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._default = oracle.lib()  # the same (unbroken) long-double F_k
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_python_mutant(name, workdir):
    mod = _load_mutant(name, workdir)
    caught = []
    for check in pins.ALL_CHECKS:
        try:
            check(mod)
        except (AssertionError, ValueError, IndexError, FloatingPointError, ZeroDivisionError) as e:
            caught.append(f"{check.__name__}: {str(e)[:80]}")
    assert caught, f"no composition pin caught mutant {name}"
