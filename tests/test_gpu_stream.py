"""A caller's HIP stream (svt_params.stream) on the GPU.

The stream comes from the HIP runtime the library links (`libamdhip64.so.7`,
looked up through the loader, so the copy already in the process): a
process can hold a second HIP runtime (PyTorch ships its own), whose stream
handles are not valid in this one.  A solve on the caller's stream gives the
same result, bit for bit, as one on the library's own stream; the library
leaves the caller's stream alive when the handle is destroyed.
"""
import ctypes

import numpy as np
import pytest

import workload
from paper_0810_3286_amd import svt as B
from tests.helpers import gpu_case

pytestmark = pytest.mark.gpu


def _solve(p, precision, stream):
    prm = B.svt_params_default(p.m, p.n, p.nnz)
    prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, p.delta, p.eps, p.maxiter, p.incr
    prm.precision = precision
    prm.stream = stream
    h = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
    try:
        st, info = B.svt_solve(h)
        U, w, V = B.svt_factors(h, p.m, p.n)
        hist = B.svt_history(h)
    finally:
        B.svt_destroy(h)
    return st, info, U, w, V, hist


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
def test_caller_stream_gives_the_same_solve(precision):
    gpu_case(f"caller stream, 400^2 solve, precision {precision}")
    hip = ctypes.CDLL("libamdhip64.so.7")
    s = ctypes.c_void_p()
    assert hip.hipStreamCreate(ctypes.byref(s)) == 0          # default priority
    try:
        p = workload.config(1)
        a = _solve(p, precision, None)
        b = _solve(p, precision, s.value)
        assert a[0] == b[0] == B.SVT_OK
        assert a[1].iters == b[1].iters and a[1].rank == b[1].rank
        for x, y in zip(a[2:5], b[2:5]):
            np.testing.assert_array_equal(x, y)
        np.testing.assert_array_equal(a[5]["residuals"], b[5]["residuals"])
        # the caller's stream outlives the handle
        assert hip.hipStreamSynchronize(s) == 0
    finally:
        assert hip.hipStreamDestroy(s) == 0
