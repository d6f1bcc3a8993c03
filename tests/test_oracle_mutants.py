"""Plant plausible mistakes in the oracle (on the CPU) and require the pins to
catch every one: a dropped term, a wrong sign, an index off by one, a
transposed operand, a loose stopping rule, a misplaced branch switch."""
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle
from tests import oracle_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "boys_oracle.c")

MUTANTS = {
    "series_index_off_by_one": ("term *= x / (K + (long double)l + 0.5L);",
                                "term *= x / (K + (long double)l + 1.5L);"),
    "series_first_term_dropped": ("long double sum = term;", "long double sum = 0.0L;"),
    "series_prefactor_dropped": ("F[kmax] = 0.5L * emx * sum;", "F[kmax] = emx * sum;"),
    "series_operand_transposed": ("term *= x / (K + (long double)l + 0.5L);",
                                  "term *= (K + (long double)l + 0.5L) / x;"),
    "stopping_rule_loose": ("ldexpl(fabsl(sum), -72)", "ldexpl(fabsl(sum), -30)"),
    "downward_exp_term_dropped": ("F[k] = (2.0L * x * F[k + 1] + emx) / (2.0L * k + 1.0L);",
                                  "F[k] = (2.0L * x * F[k + 1]) / (2.0L * k + 1.0L);"),
    "downward_divisor_index": ("F[k] = (2.0L * x * F[k + 1] + emx) / (2.0L * k + 1.0L);",
                               "F[k] = (2.0L * x * F[k + 1] + emx) / (2.0L * k + 3.0L);"),
    "upward_sign_flipped": ("F[k + 1] = ((2.0L * k + 1.0L) * F[k] - emx) / (2.0L * x);",
                            "F[k + 1] = ((2.0L * k + 1.0L) * F[k] + emx) / (2.0L * x);"),
    "upward_factor_index": ("F[k + 1] = ((2.0L * k + 1.0L) * F[k] - emx) / (2.0L * x);",
                            "F[k + 1] = ((2.0L * k + 3.0L) * F[k] - emx) / (2.0L * x);"),
    "closed_form_sqrt_dropped": ("F[0] = 0.5L * sqrtl(pi / x) * erfl(s);",
                                 "F[0] = 0.5L * (pi / x) * erfl(s);"),
    "closed_form_erf_argument": ("F[0] = 0.5L * sqrtl(pi / x) * erfl(s);",
                                 "F[0] = 0.5L * sqrtl(pi / x) * erfl(x);"),
    "branch_switch_too_low": ("#define SERIES_MAX 30.0L", "#define SERIES_MAX 3.0L"),
    "exp_sign": ("const long double emx = expl(-x);", "const long double emx = expl(x);"),
}


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="oracle_mutants_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, workdir):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not found exactly once"
    src = os.path.join(workdir, f"{name}.c")
    lib = os.path.join(workdir, f"lib{name}.so")
    with open(src, "w") as f:
        f.write(text.replace(old, new))
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", lib, src, "-lm"], check=True)
    o = oracle.OracleLib(lib)
    caught = []
    for check in oracle_pins.ALL_CHECKS:
        try:
            check(o)
        except (AssertionError, ValueError, FloatingPointError, OverflowError, ZeroDivisionError) as e:
            caught.append(f"{check.__name__}: {str(e)[:80]}")
    assert caught, f"no pin caught mutant {name}"
