"""ctypes binding of the C ABI in ``include/svt.h`` (argument marshalling only).

Every function here has the name of the C entry point it calls; all numerical
work happens in the HIP library.  Loading fails loudly when the library has not
been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libsvt.so")

SVT_OK = 0
SVT_NOT_CONVERGED = 1
SVT_STALLED = 2
SVT_UNDERDETERMINED = 3
SVT_EINVAL = -1
SVT_ENOMEM = -2
SVT_EDEVICE = -3
SVT_ESTATE = -4
SVT_EDIVERGED = -5
SVT_EBUSY = -6
SVT_ELANCZOS = -7

SVT_FP64 = 0
SVT_MIXED = 1
SVT_COO = 0
SVT_CSR = 1
SVT_STOP_RELRES = 0
SVT_STOP_NOISY = 1
SVT_CONSTRAINT_EQUALITY = 0
SVT_CONSTRAINT_INEQUALITY = 1
SVT_SVD_LANCZOS = 0
SVT_SVD_RANDOMIZED = 1

KERNEL_KINDS = {0: "k_spmv", 1: "k_gather", 2: "k_gs_update_pass1", 3: "k_ritz", 4: "k_sample_update",
                5: "k_gs_update_pass2", 6: "k_pending_reduce"}


class svt_params(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("maxiter", ctypes.c_int32),
        ("incr", ctypes.c_int32),
        ("kick", ctypes.c_int32),
        ("k0_override", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("stop_rule", ctypes.c_int32),
        ("noise_sigma", ctypes.c_double),
        ("lanczos_tol", ctypes.c_double),
        ("lanczos_maxsteps", ctypes.c_int32),
        ("reorth_passes", ctypes.c_int32),
        ("decide_margin", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("profile", ctypes.c_int32),
        ("spmv_mode", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("ineq_tol", ctypes.c_double),
        ("constraint", ctypes.c_int32),
        ("warm_start", ctypes.c_int32),
        ("stall_window", ctypes.c_int32),
        ("min_block_rows", ctypes.c_int32),
        ("svd_method", ctypes.c_int32),
        ("rsvd_oversample", ctypes.c_int32),
        ("rsvd_power", ctypes.c_int32),
        ("reorth_eta", ctypes.c_double),
        ("dof_bound", ctypes.c_double),
    ]


class svt_info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("k0", ctypes.c_int32),
        ("rank", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("rel_residual", ctypes.c_double),
        ("sigma1", ctypes.c_double),
        ("norm_pm", ctypes.c_double),
        ("t_setup_s", ctypes.c_double),
        ("t_kick_s", ctypes.c_double),
        ("t_solve_s", ctypes.c_double),
        ("gkl_steps", ctypes.c_int64),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class SvtError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status
        self.info = None


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)


def _signatures(lib):
    h = ctypes.c_void_p
    sig = {
        "svt_params_default": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                                ctypes.POINTER(svt_params)]),
        "svt_create": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_void_p, _ip, _dp, ctypes.POINTER(svt_params),
                                        ctypes.POINTER(ctypes.c_void_p)]),
        "svt_create_sensing": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _ip, _ip,
                                                ctypes.c_int64, _lp, _ip, _dp, _dp, ctypes.POINTER(svt_params),
                                                ctypes.POINTER(ctypes.c_void_p)]),
        "svt_solve": (ctypes.c_int32, [h, ctypes.POINTER(svt_info)]),
        "svt_solve_path": (ctypes.c_int32, [h, _dp, ctypes.c_int32, ctypes.POINTER(svt_info)]),
        "svt_history": (ctypes.c_int32, [h, ctypes.c_int32, _ip, _ip, _dp, _ip, _ip]),
        "svt_factors": (ctypes.c_int32, [h, _ip, _dp, _dp, _dp]),
        "svt_predict": (ctypes.c_int32, [h, ctypes.c_int64, _ip, _ip, _dp]),
        "svt_destroy": (None, [h]),
        "svt_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
        "svt_last_error": (ctypes.c_char_p, [h]),
        "svt_set_iterate": (ctypes.c_int32, [h, _dp]),
        "svt_get_iterate": (ctypes.c_int32, [h, ctypes.c_int32, _dp]),
        "svt_set_multipliers": (ctypes.c_int32, [h, _dp, _dp]),
        "svt_get_multipliers": (ctypes.c_int32, [h, _dp, _dp]),
        "svt_apply": (ctypes.c_int32, [h, ctypes.c_int32, _dp, _dp]),
        "svt_partial_svd": (ctypes.c_int32, [h, ctypes.c_int32, _dp, _dp, _dp, _ip]),
        "svt_sample_update": (ctypes.c_int32, [h, ctypes.c_int32, _dp, _dp, ctypes.c_double, _dp]),
        "svt_kick": (ctypes.c_int32, [h, _dp, _ip]),
        "svt_sample_update_noalloc": (ctypes.c_int32, [h, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                                       ctypes.c_int64, ctypes.c_double, _dp]),
        "svt_kernel_stats": (ctypes.c_int32, [h, ctypes.c_int32, _lp, _dp, _dp]),
        "svt_reorth_stats": (ctypes.c_int32, [h, _lp, _lp, _lp, _lp]),
        "svt_spmv_plan": (ctypes.c_int32, [h, ctypes.c_int32, _ip]),
        "svt_device_bytes": (ctypes.c_int32, [h, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
        "svt_footprint": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_size_t)]),
        "svt_server_create": (ctypes.c_int32, [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
        "svt_submit": (ctypes.c_int32, [h, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _ip, _ip, _dp,
                                        ctypes.POINTER(svt_params), ctypes.POINTER(ctypes.c_uint64)]),
        "svt_poll": (ctypes.c_int32, [h, ctypes.c_uint64, _ip]),
        "svt_wait": (ctypes.c_int32, [h, ctypes.c_uint64, ctypes.POINTER(svt_info)]),
        "svt_result": (ctypes.c_int32, [h, ctypes.c_uint64, _ip, _dp, _dp, _dp, _dp]),
        "svt_release": (ctypes.c_int32, [h, ctypes.c_uint64]),
        "svt_server_stats": (ctypes.c_int32, [h, ctypes.POINTER(ctypes.c_size_t), _ip, _ip]),
        "svt_server_destroy": (ctypes.c_int32, [h]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"HIP library not built: {path} is missing; run "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        _lib = _signatures(ctypes.CDLL(path))
    return _lib


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.shape[0] != n:
        raise ValueError("length mismatch")
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


def svt_status_string(status: int) -> str:
    return load().svt_status_string(status).decode()


def svt_last_error(h=None) -> str:
    return load().svt_last_error(h).decode()


def _check(status, h=None, allow=(SVT_OK,)):
    if status not in allow:
        raise SvtError(status, f"{svt_status_string(status)}: {svt_last_error(h)}")
    return status


def svt_params_default(m: int, n: int, nnz: int) -> svt_params:
    p = svt_params()
    _check(load().svt_params_default(m, n, nnz, ctypes.byref(p)))
    return p


def svt_create(m: int, n: int, rows, cols, vals, params: svt_params | None = None,
               fmt: int = SVT_COO):
    """Create a problem from COO triplets (or CSR: rows = int64 rowptr[m+1])."""
    lib = load()
    cols = _i32(cols)
    vals = _f64(vals)
    nnz = cols.shape[0]
    if fmt == SVT_CSR:
        idx0 = np.ascontiguousarray(rows, dtype=np.int64)
    else:
        idx0 = _i32(rows)
    if vals.shape[0] != nnz or (fmt == SVT_COO and idx0.shape[0] != nnz):
        raise ValueError("rows, cols and vals must have the same length")
    h = ctypes.c_void_p()
    st = lib.svt_create(m, n, nnz, fmt, idx0.ctypes.data_as(ctypes.c_void_p), _p(cols, _ip), _p(vals),
                        ctypes.byref(params) if params is not None else None, ctypes.byref(h))
    _check(st, None)
    return h


def svt_create_sensing(m: int, n: int, srows, scols, gptr, gidx, gval, b, params: svt_params | None = None):
    """Create a problem with a general linear operator: support positions
    (srows, scols) and the measurement matrix in CSR form (gptr int64[p+1],
    gidx into the support, gval), measurements b."""
    srows = _i32(srows)
    scols = _i32(scols)
    gptr = np.ascontiguousarray(gptr, dtype=np.int64)
    gidx = _i32(gidx)
    gval = _f64(gval)
    b = _f64(b)
    h = ctypes.c_void_p()
    st = load().svt_create_sensing(m, n, srows.shape[0], _p(srows, _ip), _p(scols, _ip), b.shape[0],
                                   _p(gptr, _lp), _p(gidx, _ip), _p(gval), _p(b),
                                   ctypes.byref(params) if params is not None else None, ctypes.byref(h))
    _check(st, None)
    return h


def svt_destroy(h) -> None:
    if h is not None:
        load().svt_destroy(h)


def svt_solve(h):
    """Returns (status, info) for SVT_OK / SVT_NOT_CONVERGED / SVT_STALLED /
    SVT_UNDERDETERMINED; raises SvtError
    otherwise, with the info of the iterations completed as ``.info``."""
    info = svt_info()
    st = load().svt_solve(h, ctypes.byref(info))
    try:
        _check(st, h, allow=(SVT_OK, SVT_NOT_CONVERGED, SVT_STALLED, SVT_UNDERDETERMINED))
    except SvtError as e:
        e.info = info
        raise
    return st, info


def svt_solve_path(h, taus):
    """tau continuation: returns (status, [info per stage]); raises SvtError
    on an error, with the stages done as ``.info``."""
    taus = _f64(taus)
    infos = (svt_info * taus.shape[0])()
    st = load().svt_solve_path(h, _p(taus), taus.shape[0], infos)
    try:
        _check(st, h, allow=(SVT_OK, SVT_NOT_CONVERGED, SVT_STALLED, SVT_UNDERDETERMINED))
    except SvtError as e:
        e.info = list(infos)
        raise
    return st, list(infos)


def svt_history(h):
    lib = load()
    ln = ctypes.c_int32()
    _check(lib.svt_history(h, 0, None, None, None, None, ctypes.byref(ln)), h)
    n = ln.value
    ranks = np.zeros(n, np.int32)
    s = np.zeros(n, np.int32)
    res = np.zeros(n, np.float64)
    steps = np.zeros(n, np.int32)
    _check(lib.svt_history(h, n, _p(ranks, _ip), _p(s, _ip), _p(res), _p(steps, _ip),
                           ctypes.byref(ln)), h)
    return dict(ranks=ranks, s_hist=s, residuals=res, gkl_steps=steps)


def svt_factors(h, m: int, n: int):
    lib = load()
    r = ctypes.c_int32()
    _check(lib.svt_factors(h, ctypes.byref(r), None, None, None), h)
    r = r.value
    U = np.zeros((m, r))
    V = np.zeros((n, r))
    w = np.zeros(r)
    if r > 0:
        rr = ctypes.c_int32()
        _check(lib.svt_factors(h, ctypes.byref(rr), _p(U), _p(w), _p(V)), h)
    return U, w, V


def svt_predict(h, rows, cols):
    rows = _i32(rows)
    cols = _i32(cols)
    out = np.zeros(rows.shape[0])
    _check(load().svt_predict(h, rows.shape[0], _p(rows, _ip), _p(cols, _ip), _p(out)), h)
    return out


def svt_set_iterate(h, y):
    y = _f64(y)
    _check(load().svt_set_iterate(h, _p(y)), h)


def svt_get_iterate(h, nnz: int, which: int = 0):
    y = np.zeros(nnz)
    _check(load().svt_get_iterate(h, which, _p(y)), h)
    return y


def svt_set_multipliers(h, yp, ym):
    yp = _f64(yp)
    ym = _f64(ym, yp.shape[0])
    _check(load().svt_set_multipliers(h, _p(yp), _p(ym)), h)


def svt_get_multipliers(h, nnz: int):
    yp = np.zeros(nnz)
    ym = np.zeros(nnz)
    _check(load().svt_get_multipliers(h, _p(yp), _p(ym)), h)
    return yp, ym


def svt_apply(h, x, out_len: int, trans: int = 0):
    x = _f64(x)
    out = np.zeros(out_len)
    _check(load().svt_apply(h, trans, _p(x), _p(out)), h)
    return out


def svt_partial_svd(h, count: int, m: int, n: int):
    sigma = np.zeros(count)
    U = np.zeros((m, count))
    V = np.zeros((n, count))
    steps = ctypes.c_int32()
    _check(load().svt_partial_svd(h, count, _p(sigma), _p(U), _p(V), ctypes.byref(steps)), h)
    return sigma, U, V, steps.value


def svt_sample_update(h, U, V, delta: float) -> float:
    U = np.ascontiguousarray(U, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    r = U.shape[1] if U.ndim == 2 else 0
    res2 = ctypes.c_double()
    _check(load().svt_sample_update(h, r, _p(U), _p(V), float(delta), ctypes.byref(res2)), h)
    return res2.value


def svt_sample_update_noalloc(h, r: int, U_dev: int, V_dev: int, stride: int, delta: float) -> float:
    """svt_sample_update with device-resident factors (integer device
    addresses, the handle's value type, row stride ``stride``); allocates
    nothing."""
    res2 = ctypes.c_double()
    _check(load().svt_sample_update_noalloc(h, r, ctypes.c_void_p(U_dev), ctypes.c_void_p(V_dev), stride,
                                            float(delta), ctypes.byref(res2)), h)
    return res2.value


def svt_kick(h):
    s = ctypes.c_double()
    k0 = ctypes.c_int32()
    _check(load().svt_kick(h, ctypes.byref(s), ctypes.byref(k0)), h)
    return s.value, k0.value


def svt_kernel_stats(h, kind: int):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    b = ctypes.c_double()
    _check(load().svt_kernel_stats(h, kind, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)), h)
    return n.value, ms.value, b.value


def svt_reorth_stats(h):
    """(vectors made, vectors orthogonalised against their basis, restarts
    with two Gram-Schmidt passes, fallbacks from partial to full
    reorthogonalisation) of the handle's last solve."""
    v = [ctypes.c_int64() for _ in range(4)]
    _check(load().svt_reorth_stats(h, *[ctypes.byref(x) for x in v]), h)
    return tuple(x.value for x in v)


def svt_spmv_plan(h, which: int) -> int:
    """Column segments of x staged in LDS by the row- (0) or column-compressed
    (1) sparse product; 0 when it gathers x from memory."""
    seg = ctypes.c_int32()
    _check(load().svt_spmv_plan(h, which, ctypes.byref(seg)), h)
    return seg.value


def svt_device_bytes(h):
    """(bytes held now, most bytes held at once) of a handle's device memory."""
    cur = ctypes.c_size_t()
    peak = ctypes.c_size_t()
    _check(load().svt_device_bytes(h, ctypes.byref(cur), ctypes.byref(peak)), h)
    return cur.value, peak.value


# ---------------------------------------------------------------- serving


def svt_footprint(m: int, n: int, nnz: int, precision: int = SVT_FP64) -> int:
    b = ctypes.c_size_t()
    _check(load().svt_footprint(m, n, nnz, precision, ctypes.byref(b)))
    return b.value


def svt_server_create(hbm_budget_bytes: int, max_slots: int):
    s = ctypes.c_void_p()
    _check(load().svt_server_create(hbm_budget_bytes, max_slots, ctypes.byref(s)))
    return s


def svt_submit(server, m: int, n: int, rows, cols, vals, params: svt_params | None = None) -> int:
    rows = _i32(rows)
    cols = _i32(cols)
    vals = _f64(vals)
    if not (rows.shape[0] == cols.shape[0] == vals.shape[0]):
        raise ValueError("rows, cols and vals must have the same length")
    t = ctypes.c_uint64()
    st = load().svt_submit(server, m, n, vals.shape[0], _p(rows, _ip), _p(cols, _ip), _p(vals),
                           ctypes.byref(params) if params is not None else None, ctypes.byref(t))
    if st != SVT_OK:
        raise SvtError(st, svt_status_string(st))
    return t.value


def svt_poll(server, ticket: int) -> int:
    st = ctypes.c_int32()
    _check(load().svt_poll(server, ticket, ctypes.byref(st)))
    return st.value


def svt_wait(server, ticket: int):
    info = svt_info()
    st = load().svt_wait(server, ticket, ctypes.byref(info))
    return st, info


def svt_result(server, ticket: int, m: int, n: int):
    lib = load()
    r = ctypes.c_int32()
    st = lib.svt_result(server, ticket, ctypes.byref(r), None, None, None, None)
    if st == SVT_EINVAL or st == SVT_EBUSY:
        raise SvtError(st, svt_status_string(st))
    # a failed solve still carries its timestamps (and rank 0)
    r = r.value if st in (SVT_OK, SVT_NOT_CONVERGED, SVT_STALLED, SVT_UNDERDETERMINED) else 0
    U = np.zeros((m, r))
    V = np.zeros((n, r))
    w = np.zeros(r)
    times = np.zeros(3)
    rr = ctypes.c_int32()
    lib.svt_result(server, ticket, ctypes.byref(rr), _p(U), _p(w), _p(V), _p(times))
    return st, U, w, V, times


def svt_release(server, ticket: int) -> None:
    _check(load().svt_release(server, ticket))


def svt_server_stats(server):
    b = ctypes.c_size_t()
    mr = ctypes.c_int32()
    q = ctypes.c_int32()
    _check(load().svt_server_stats(server, ctypes.byref(b), ctypes.byref(mr), ctypes.byref(q)))
    return dict(peak_bytes=b.value, max_running=mr.value, queued=q.value)


def svt_server_destroy(server) -> None:
    if server is not None:
        load().svt_server_destroy(server)
