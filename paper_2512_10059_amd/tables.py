"""Read the degree tables of the library's coefficient headers (host side).

Used for operation counts in reports; the kernels take the coefficients
from the headers at compile time."""
from __future__ import annotations

import os
import re

_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def _define(path: str, name: str) -> str:
    text = open(path).read().replace("\\\n", " ")
    m = re.search(r"^#define\s+" + name + r"\s+(.*)$", text, re.M)
    if not m:
        raise KeyError(name)
    return m.group(1)


def f64_region_a_degrees():
    """[(n_k, m_k)] numerator/denominator degrees of r_{A,k}, k = 0..32."""
    h = os.path.join(_CSRC, "boys_coeffs_f64.h")
    n = [int(v) for v in re.findall(r"-?\d+", _define(h, "BOYS_RA_DEG_N_INIT"))]
    m = [int(v) for v in re.findall(r"-?\d+", _define(h, "BOYS_RA_DEG_M_INIT"))]
    return list(zip(n, m))


def f32_region_bounds():
    """(x0', x1') of the FP32 path, as the kernels hold them (FP32 values):
    A' = [0, x0'), B' = [x0', x1'), C' = [x1', inf)."""
    h = os.path.join(_CSRC, "boys_coeffs_f32.h")
    return tuple(float.fromhex(_define(h, name).strip().rstrip("f")) for name in ("BOYS_F32_X0", "BOYS_F32_X1"))
