"""MI355X (gfx950) singular value thresholding for matrix completion.

The numerical path lives in the HIP library built from ``csrc/`` (C ABI in
``include/svt.h``); ``svt`` is its ctypes binding.  ``solve`` is a small
convenience wrapper over create / solve / factors / destroy.
"""
from __future__ import annotations

from . import svt  # noqa: F401
from .svt import (  # noqa: F401
    SVT_COO, SVT_CSR, SVT_FP64, SVT_MIXED, SVT_NOT_CONVERGED, SVT_OK, SVT_STOP_NOISY,
    SVT_STOP_RELRES, SvtError, svt_apply, svt_create, svt_destroy, svt_factors, svt_get_iterate,
    svt_history, svt_kernel_stats, svt_kick, svt_last_error, svt_params, svt_params_default,
    svt_partial_svd, svt_predict, svt_sample_update, svt_set_iterate, svt_solve,
    svt_status_string,
)


def solve(m, n, rows, cols, vals, **params):
    """Create, solve, read the factors and destroy.  Keyword arguments set
    fields of ``svt_params`` (defaults from ``svt_params_default``)."""
    p = svt_params_default(m, n, len(vals))
    for k, v in params.items():
        setattr(p, k, v)
    h = svt_create(m, n, rows, cols, vals, p)
    try:
        status, info = svt_solve(h)
        U, w, V = svt_factors(h, m, n)
        hist = svt_history(h)
        reorth = svt.svt_reorth_stats(h)
    finally:
        svt_destroy(h)
    return dict(status=status, info=info.as_dict(), U=U, w=w, V=V, reorth=reorth, **hist)
