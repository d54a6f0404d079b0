"""The allocation-free sampled pass (svt_sample_update_noalloc) against the
existing entry point (svt_sample_update) through the C ABI: the same
residual and the same iterate in both compressed copies, bit for bit, on two
calls in a row (the second on a smaller problem, reusing the device's fixed
scratch), in both precisions; the handle's device memory does not change
during the call, and bad strides are refused before any device work."""
import ctypes

import numpy as np
import pytest

import workload
from paper_0810_3286_amd import svt as B
from tests.helpers import gpu_case

pytestmark = pytest.mark.gpu

CASES = [(900, 700, 12, 60000, 3), (300, 250, 5, 9000, 4)]   # the second is smaller


class _DeviceBuffer:
    """A caller-owned device buffer made through the HIP runtime the library
    itself links (one runtime per process), holding F padded to `stride`
    columns in the handle's value type."""

    def __init__(self, F, stride, dtype):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        host = np.zeros((F.shape[0], stride), dtype=dtype)
        host[:, :F.shape[1]] = F
        self.nbytes = host.nbytes
        self.ptr = ctypes.c_void_p()
        assert self.hip.hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(self.nbytes)) == 0
        assert self.hip.hipMemcpy(self.ptr, host.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.c_size_t(self.nbytes), 1) == 0   # host to device
        assert self.hip.hipDeviceSynchronize() == 0

    def free(self):
        if self.ptr:
            self.hip.hipFree(self.ptr)
            self.ptr = ctypes.c_void_p()


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
def test_noalloc_equals_sample_update_twice(precision):
    dtype = np.float64 if precision == B.SVT_FP64 else np.float32
    al = 2 if precision == B.SVT_FP64 else 4
    for case in CASES:
        gpu_case(f"no-alloc sampled pass {case} precision {precision}")
        p = workload.gaussian_lowrank(*case)
        r = p.r
        rng = np.random.default_rng(7 + r)
        y0 = rng.standard_normal(p.nnz) * 3.0
        U = rng.standard_normal((p.m, r))
        V = rng.standard_normal((p.n, r))
        delta = 1.7
        prm = B.svt_params_default(p.m, p.n, p.nnz)
        prm.precision = precision
        ha = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
        hb = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
        Ud = Vd = None
        try:
            B.svt_set_iterate(ha, y0)
            B.svt_set_iterate(hb, y0)
            res_a = B.svt_sample_update(ha, U, V, delta)
            stride = (r + al - 1) // al * al + al   # wider than r: the stride is honoured
            Ud = _DeviceBuffer(U, stride, dtype)
            Vd = _DeviceBuffer(V, stride, dtype)
            before, _ = B.svt_device_bytes(hb)
            res_b = B.svt_sample_update_noalloc(hb, r, Ud.ptr.value, Vd.ptr.value, stride, delta)
            after, _ = B.svt_device_bytes(hb)
            assert after == before
            assert res_b == res_a
            for which in (0, 1):
                np.testing.assert_array_equal(B.svt_get_iterate(hb, p.nnz, which),
                                              B.svt_get_iterate(ha, p.nnz, which))
            # refused on the host: a stride below r, and one that is not a
            # multiple of 16 bytes
            for bad in (r - 1, stride + 1):
                with pytest.raises(B.SvtError):
                    B.svt_sample_update_noalloc(hb, r, Ud.ptr.value, Vd.ptr.value, bad, delta)
        finally:
            B.svt_destroy(ha)
            B.svt_destroy(hb)
            for d in (Ud, Vd):
                if d is not None:
                    d.free()
