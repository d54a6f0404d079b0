"""The C ABI library (CPU only: loading, exports and argument validation).

Validation runs before any device call, so every rejection below is checked
without a GPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_0810_3286_amd import svt as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def _declared():
    names = set()
    for fn in os.listdir(HEADER_DIR):
        if fn.endswith(".h"):
            txt = open(os.path.join(HEADER_DIR, fn)).read()
            names |= set(re.findall(r"^\s*(?:svt_status|void|const char \*)\s*(svt_\w+)\s*\(", txt, re.M))
    return names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(B.LIB_PATH)
    names = _declared()
    assert len(names) >= 16
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_binding_covers_every_declared_symbol():
    names = _declared()
    assert all(hasattr(B, n) for n in names), sorted(n for n in names if not hasattr(B, n))


def test_randomized_svd_refused_outside_completion():
    rows = np.array([0, 1], dtype=np.int32)
    cols = np.array([0, 1], dtype=np.int32)
    vals = np.array([1.0, 2.0])
    p = B.svt_params_default(2, 2, 2)
    p.svd_method = B.SVT_SVD_RANDOMIZED
    p.constraint = B.SVT_CONSTRAINT_INEQUALITY
    _expect_einval(2, 2, rows, cols, vals, p)


def test_struct_layout_matches_header():
    # svt_params: 3 doubles, 6 int32, 2 doubles, 2 int32, double, uint64, 2 int32, pointer,
    # double, 7 int32 (and 4 bytes of padding), 2 doubles
    assert ctypes.sizeof(B.svt_params) == 3 * 8 + 6 * 4 + 2 * 8 + 2 * 4 + 8 + 8 + 2 * 4 + 8 + 8 + 7 * 4 + 4 + 16
    assert B.svt_params.reorth_eta.offset == ctypes.sizeof(B.svt_params) - 16
    assert B.svt_params.dof_bound.offset == ctypes.sizeof(B.svt_params) - 8
    assert ctypes.sizeof(B.svt_info) == 4 * 4 + 6 * 8 + 8


def test_params_default_is_the_papers_choice():
    p = B.svt_params_default(400, 400, 47400)
    assert p.tau == pytest.approx(2000.0)
    assert p.delta == pytest.approx(1.2 * 400 * 400 / 47400)
    assert p.eps == 1e-4 and p.maxiter == 500 and p.incr == 5 and p.kick == 1
    # partial reorthogonalisation, as the paper's PROPACK runs (Section 5.1.1)
    assert p.reorth_eta < 0          # automatic: 0.01 sqrt(u) FP64, 0.1 sqrt(u) FP32
    q = B.svt_params_default(300, 1200, 1000)
    assert q.tau == pytest.approx(5.0 * np.sqrt(300 * 1200))
    with pytest.raises(B.SvtError):
        B.svt_params_default(0, 5, 5)


def test_status_strings():
    for s in (0, 1, 2, 3, -1, -2, -3, -4, -5, -6, -7):
        assert B.svt_status_string(s)
    assert "unknown" in B.svt_status_string(99)


def _expect_einval(*args, match=None, **kw):
    with pytest.raises(B.SvtError) as e:
        B.svt_create(*args, **kw)
    assert e.value.status == B.SVT_EINVAL
    if match:
        assert match in str(e.value)


def test_rejects_bad_shapes_and_indices():
    rows = np.array([0, 1, 2], np.int32)
    cols = np.array([0, 1, 2], np.int32)
    vals = np.array([1.0, 2.0, 3.0])
    _expect_einval(0, 3, rows, cols, vals, match="m and n")
    _expect_einval(3, 3, np.array([0, 1, 3], np.int32), cols, vals, match="row index")
    _expect_einval(3, 3, rows, np.array([0, -1, 2], np.int32), vals, match="column index")
    _expect_einval(3, 3, np.array([0, 1, 1], np.int32), np.array([0, 2, 2], np.int32), vals,
                   match="duplicate")
    _expect_einval(3, 3, rows, cols, np.array([1.0, np.nan, 3.0]), match="non-finite")
    _expect_einval(3, 3, rows, cols, np.zeros(3), match="zero")
    _expect_einval(1, 2, np.zeros(3, np.int32), np.array([0, 1, 1], np.int32), vals)


def test_rejects_bad_parameters():
    rows = np.array([0, 1], np.int32)
    cols = np.array([0, 1], np.int32)
    vals = np.array([1.0, 2.0])
    for field, bad in [("tau", 0.0), ("tau", float("inf")), ("delta", -1.0), ("eps", -1e-3),
                       ("maxiter", 0), ("incr", 0), ("kick", 2), ("precision", 5),
                       ("stop_rule", 3), ("lanczos_tol", 1.5), ("reorth_passes", 3),
                       ("decide_margin", -0.1), ("spmv_mode", 3), ("min_block_rows", -1),
                       ("min_block_rows", 2049), ("svd_method", 2), ("rsvd_oversample", -1),
                       ("rsvd_power", 65), ("reorth_eta", 101.0),
                       ("reorth_eta", float("nan")), ("dof_bound", float("nan")),
                       ("dof_bound", float("inf"))]:
        p = B.svt_params_default(2, 2, 2)
        setattr(p, field, bad)
        _expect_einval(2, 2, rows, cols, vals, p)
    p = B.svt_params_default(2, 2, 2)
    p.stop_rule = B.SVT_STOP_NOISY
    _expect_einval(2, 2, rows, cols, vals, p, match="noise_sigma")


def test_rejects_bad_csr():
    cols = np.array([0, 1], np.int32)
    vals = np.array([1.0, 2.0])
    _expect_einval(2, 2, np.array([0, 1, 3], np.int64), cols, vals, fmt=B.SVT_CSR)
    _expect_einval(2, 2, np.array([0, 2, 1], np.int64), cols, vals, fmt=B.SVT_CSR)


def test_null_handle_calls_fail_cleanly():
    lib = B.load()
    assert lib.svt_solve(None, None) == B.SVT_EINVAL
    assert lib.svt_factors(None, None, None, None, None) == B.SVT_EINVAL
    lib.svt_destroy(None)
