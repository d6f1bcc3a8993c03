"""The C-ABI library loads and exports every entry point its header declares;
argument errors are rejected on the host before any HIP call (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "boys.h")
LIB = os.path.join(ROOT, "paper_2512_10059_amd", "libboys.so")

EINVAL = -1


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"BOYS_API\s+[\w\s\*]*?\b(boys_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    assert os.path.exists(LIB), "libboys.so not built"
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("boys_eval_f64", "boys_eval_f32", "boys_weighted_sum", "boys_backward",
              "boys_tune_weighted_sum", "boys_strerror", "boys_finalize"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_only_declared_symbols_are_exported():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert exported == declared()


def test_strerror(lib):
    lib.boys_strerror.restype = ctypes.c_char_p
    assert lib.boys_strerror(0) == b"success"
    assert b"invalid" in lib.boys_strerror(EINVAL)
    assert lib.boys_strerror(-99) == b"unknown status"


def test_argument_errors_without_gpu(lib):
    P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    f = lib.boys_eval_f64
    f.argtypes = [P, I64, I, P, I64, P]
    dummy = P(4096)
    assert f(dummy, -1, 8, dummy, 9, None) == EINVAL       # n < 0
    assert f(dummy, 10, 41, dummy, 42, None) == EINVAL     # kmax > 40
    assert f(dummy, 10, -1, dummy, 9, None) == EINVAL      # kmax < 0
    assert f(dummy, 10, 8, dummy, 8, None) == EINVAL       # ld_out < kmax+1
    assert f(None, 10, 8, dummy, 9, None) == EINVAL        # null x
    assert f(P(8), 10, 8, P(8), 9, None) == EINVAL         # x overlaps out
    assert f(dummy, 0, 8, None, 9, None) == 0              # empty: nothing to do
    g = lib.boys_eval_f32
    g.argtypes = [P, I64, I, P, I64, P]
    assert g(dummy, 10, 17, dummy, 18, None) == EINVAL     # FP32 tables stop at 16
    assert g(dummy, 0, 16, None, 17, None) == 0
    b = lib.boys_backward
    b.argtypes = [P, P, I64, I, I64, P, P]
    assert b(dummy, dummy, 10, 40, 41, dummy, None) == EINVAL  # needs F_41
    assert b(dummy, dummy, 10, 5, 5, dummy, None) == EINVAL    # ld_g < kmax+1
    assert b(dummy, dummy, 0, 5, 6, dummy, None) == 0
    w = lib.boys_weighted_sum
    w.argtypes = [P] * 6 + [ctypes.c_int32, P, P]
    assert w(*([dummy] * 6), -1, dummy, None) == EINVAL
    assert w(*([dummy] * 6), (1 << 24) + 1, dummy, None) == EINVAL
    assert w(None, *([dummy] * 5), 3, dummy, None) == EINVAL
    assert w(*([None] * 6), 0, None, None) == 0
    na = lib.boys_weighted_sum_noalloc
    na.argtypes = [P] * 6 + [ctypes.c_int32, P, P]
    assert na(*([dummy] * 6), 65536 + 1, dummy, None) == EINVAL  # beyond its fixed scratch
    assert na(*([dummy] * 6), -1, dummy, None) == EINVAL
    assert na(None, *([dummy] * 5), 3, dummy, None) == EINVAL
    assert na(*([None] * 6), 0, None, None) == 0
    lib.boys_weighted_sum_set_config.argtypes = [I]
    assert lib.boys_weighted_sum_set_config(999) == EINVAL
    assert lib.boys_weighted_sum_num_configs() > 1


def test_tolerance_argument_errors_without_gpu(lib):
    """The accuracy-selecting entry points reject tolerances no table set
    meets (below 5e-14, or NaN) before touching the GPU; an empty call with
    a valid tolerance succeeds without a device."""
    P, I64, I, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    f = lib.boys_eval_f64_tol
    f.argtypes = [P, I64, I, D, P, I64, P]
    dummy = P(4096)
    for tol in (4.9e-14, 0.0, -1.0, float("nan")):
        assert f(dummy, 10, 8, tol, dummy, 9, None) == EINVAL
    assert f(dummy, 10, 41, 1e-10, dummy, 42, None) == EINVAL   # kmax > 40
    for tol in (5e-14, 1e-12, 1e-10, 1.0, float("inf")):
        assert f(dummy, 0, 8, tol, None, 9, None) == 0           # empty: nothing to do
    p = lib.boys_pairsum_tol
    p.argtypes = [P, P, I64, P, I, D, P, P]
    assert p(dummy, dummy, 10, dummy, 4, 1e-15, dummy, None) == EINVAL
    assert p(dummy, dummy, 10, dummy, 4, float("nan"), dummy, None) == EINVAL
    assert p(dummy, dummy, 0, dummy, 4, 1e-10, dummy, None) == 0
    w = lib.boys_weighted_sum_tol
    w.argtypes = [P] * 6 + [ctypes.c_int32, D, P, P]
    for tol in (1e-15, float("nan")):
        assert w(*([dummy] * 6), 3, tol, dummy, None) == EINVAL
    assert w(*([None] * 6), 0, 1e-10, None, None) == 0
    b = lib.boys_backward_tol
    b.argtypes = [P, P, I64, I, I64, D, P, P]
    for tol in (1e-15, float("nan")):
        assert b(dummy, dummy, 10, 5, 6, tol, dummy, None) == EINVAL
    assert b(dummy, dummy, 0, 5, 6, 1e-10, dummy, None) == 0


def test_table_variant_setting_without_gpu(lib):
    """boys_set_tables takes the three variants, rejects anything else without
    changing the current one, and boys_get_tables reports it (host only)."""
    lib.boys_set_tables.argtypes = [ctypes.c_int]
    assert lib.boys_get_tables() == 0  # the paper's tables by default
    for v in (1, 2, 0):
        assert lib.boys_set_tables(v) == 0
        assert lib.boys_get_tables() == v
    assert lib.boys_set_tables(2) == 0
    for bad in (-1, 3, 99):
        assert lib.boys_set_tables(bad) == EINVAL
        assert lib.boys_get_tables() == 2
    assert lib.boys_set_tables(0) == 0
