"""Boys functions F_0..F_kmax on AMD Instinct MI355X (gfx950).

A C-ABI library (``libboys.so``, hand-written HIP) implements the minimax
method of arXiv 2512.10059; this package is its thin Python binding plus the
offline coefficient tooling.  Importing the package does not load the
library: the first call does, and fails loudly if it is missing.

    import paper_2512_10059_amd as boys
    F = boys.boys_eval_f64(x, kmax)          # (n, kmax+1) FP64, x on the GPU
"""
from __future__ import annotations

_BINDING_NAMES = {
    "BoysError", "BoysFunction", "boys_eval_f64", "boys_eval_f64_tol", "boys_eval_f32", "boys_weighted_sum",
    "boys_weighted_sum_noalloc",
    "boys_tune_weighted_sum", "boys_backward", "boys_pairsum", "weighted_sum_config_name",
    "weighted_sum_num_configs", "weighted_sum_get_config", "weighted_sum_set_config",
    "finalize", "lib", "library_path", "set_tables", "get_tables", "table_variant", "TABLES_PAPER",
    "TABLES_PER_KMAX", "TABLES_CENTRE", "F64_KMAX", "F64_KMAX_EVAL", "F64_KMAX_BACKWARD", "F32_KMAX",
}


def __getattr__(name):
    if name in _BINDING_NAMES:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)


__all__ = sorted(_BINDING_NAMES)
