"""Per-kernel statistics of a profiled solve (needs an MI355X): one sparse
product kernel per bidiagonalisation half-step, one sampled pass and one
column-copy gather per iteration, the Gram-Schmidt update kernels only in
two-pass mode, and algorithmic bytes for every kernel that ran."""
import pytest

import workload
from paper_0810_3286_amd import svt as B
from tests.helpers import gpu_case

pytestmark = pytest.mark.gpu


def _profiled(p, **fields):
    prm = B.svt_params_default(p.m, p.n, p.nnz)
    for k, v in dict(tau=p.tau, delta=p.delta, eps=p.eps, maxiter=p.maxiter, incr=p.incr, profile=1,
                     **fields).items():
        setattr(prm, k, v)
    h = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
    try:
        _, info = B.svt_solve(h)
        stats = {k: B.svt_kernel_stats(h, k) for k in B.KERNEL_KINDS}
    finally:
        B.svt_destroy(h)
    return info.as_dict(), stats


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
def test_one_kernel_per_half_step(precision):
    gpu_case(f"400^2 rank 10 precision {precision}: kernel statistics, one pass")
    p = workload.config(1)
    info, st = _profiled(p, precision=precision)
    iters = info["iters"]
    n_spmv, ms_spmv, b_spmv = st[0]
    assert n_spmv > 2 * iters and ms_spmv > 0 and b_spmv > 0
    # one sampled pass and one gather of the column copy per iteration
    assert st[4][0] == st[1][0] >= iters
    assert st[1][2] > 0 and st[4][2] > 0
    # Ritz vectors: one launch per side per computed iterate
    assert st[3][0] >= 2 * iters and st[3][0] % 2 == 0
    # the update is deferred into the sparse product: no update kernels
    assert st[2][0] == 0 and st[5][0] == 0


def test_two_pass_mode_runs_update_kernels():
    gpu_case("400^2 rank 10 FP64: kernel statistics, two passes")
    p = workload.config(1)
    info, st = _profiled(p, precision=B.SVT_FP64, reorth_passes=2)
    assert st[2][0] > 0 and st[5][0] > 0
    assert st[2][2] > 0 and st[5][2] > 0


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
def test_wide_basis_partial_sums_bit_identical(precision, monkeypatch):
    # from a basis width on, a pending vector's partials are summed by their
    # own kernel before the sparse product; below it every workgroup of the
    # product sums them itself.  Moving the width (the tuning hook) must not
    # change a bit.
    gpu_case(f"300x250 partial_svd 70 triplets precision {precision}: separate partial sums on and off")
    import numpy as np
    p = workload.gaussian_lowrank(300, 250, 5, 30000, 21)
    y = workload.dense_random_iterate(p, 22)
    runs = []
    for width in ("32", "100000"):
        monkeypatch.setenv("SVT_PREREDUCE_MIN", width)
        prm = B.svt_params_default(p.m, p.n, p.nnz)
        prm.precision = precision
        prm.profile = 1
        h = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
        try:
            B.svt_set_iterate(h, y)
            sig, U, V, steps = B.svt_partial_svd(h, 70, p.m, p.n)
            n_red = B.svt_kernel_stats(h, 6)[0]
        finally:
            B.svt_destroy(h)
        runs.append((sig, U, V, steps, n_red))
    (s0, U0, V0, k0, r0), (s1, U1, V1, k1, r1) = runs
    assert k0 == k1 > 64
    assert r0 > 0 and r1 == 0
    np.testing.assert_array_equal(s0, s1)
    np.testing.assert_array_equal(U0, U1)
    np.testing.assert_array_equal(V0, V1)
