"""Serving form, host side (no GPU): request validation and admission limits
are decided before any device work."""
import numpy as np
import pytest

from paper_0810_3286_amd import svt as B


def test_footprint_grows_with_size_and_precision():
    a = B.svt_footprint(1000, 1000, 60000)
    b = B.svt_footprint(2000, 2000, 120000)
    c = B.svt_footprint(1000, 1000, 60000, B.SVT_MIXED)
    assert 0 < a < b and c < a
    with pytest.raises(B.SvtError):
        B.svt_footprint(0, 10, 10)


def test_submit_rejects_invalid_and_oversized_requests():
    srv = B.svt_server_create(1 << 20, 2)  # 1 MiB: nothing real fits
    try:
        rows = np.array([0, 1], np.int32)
        cols = np.array([0, 5], np.int32)   # column 5 out of range for n = 3
        with pytest.raises(B.SvtError) as e:
            B.svt_submit(srv, 3, 3, rows, cols, np.array([1.0, 2.0]))
        assert e.value.status == B.SVT_EINVAL
        rows = np.arange(2000, dtype=np.int32)
        cols = np.arange(2000, dtype=np.int32)
        with pytest.raises(B.SvtError) as e:
            B.svt_submit(srv, 2000, 2000, rows, cols, np.ones(2000))
        assert e.value.status == B.SVT_ENOMEM
        assert B.svt_server_stats(srv)["queued"] == 0
    finally:
        B.svt_server_destroy(srv)


def test_server_create_rejects_bad_arguments():
    with pytest.raises(B.SvtError):
        B.svt_server_create(0, 2)
    with pytest.raises(B.SvtError):
        B.svt_server_create(1 << 30, 0)
