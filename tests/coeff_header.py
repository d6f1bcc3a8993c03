"""Read the coefficient headers of the GPU library as numbers (test helper)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_10059_amd", "csrc")


def _defines(path):
    text = open(path).read().replace("\\\n", " ")
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    out = {}
    for m in re.finditer(r"^#define\s+(\w+)\s+(.*)$", text, re.M):
        out[m.group(1)] = m.group(2).strip()
    return out


def _nested(s):
    s = s.strip()
    if s.startswith("{"):
        rows = re.findall(r"\{([^{}]*)\}", s[1:-1]) if s[1:].lstrip().startswith("{") else [s[1:-1]]
        vals = [[float(v) for v in r.split(",") if v.strip()] for r in rows]
        return vals if len(vals) > 1 or s[1:].lstrip().startswith("{") else vals[0]
    return float(s)


def load_f64():
    d = _defines(os.path.join(CSRC, "boys_coeffs_f64.h"))
    degn = [int(v) for v in _nested(d["BOYS_RA_DEG_N_INIT"])]
    degm = [int(v) for v in _nested(d["BOYS_RA_DEG_M_INIT"])]
    P = _nested(d["BOYS_RA_P_INIT"])
    Q = _nested(d["BOYS_RA_Q_INIT"])
    ra = [(P[k][:degn[k] + 1], Q[k][:degm[k] + 1]) for k in range(len(degn))]
    rb = (_nested(d["BOYS_RB_P_INIT"]), _nested(d["BOYS_RB_Q_INIT"]))
    return dict(x0=float(d["BOYS_F64_X0"]), x1=float(d["BOYS_F64_X1"]), ra=ra, rb=rb,
                raw=d)
