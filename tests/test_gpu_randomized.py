"""The randomised partial SVD (Section 6's first direction, svd_method =
SVT_SVD_RANDOMIZED) on the GPU against the CPU oracle's randomised SVT
(oracle/randomized.py: the same counter-based test matrices, LAPACK's
Householder QR where the library uses Gram-Schmidt twice -- the same
subspaces, so the same triplets up to rounding):

* FP64 at a fixed iteration count: the same ranks and s_k, residual
  histories within 1e-8 and X within 1e-8, for two power-iteration counts;
* with as many test vectors as the smaller dimension the triplets are
  exact, and the whole solve matches the exact oracle (tier A);
* the mixed form within the mixed bar (5e-4);
* the library refuses it for the Dantzig selector.
"""
import numpy as np
import pytest

import oracle
import workload
from oracle.randomized import svt_randomized
from paper_0810_3286_amd import solve
from paper_0810_3286_amd import svt as B
from tests.helpers import gpu_case, rel_diff_factored

pytestmark = pytest.mark.gpu

SEED = 11


def _gpu(p, maxiter, eps, precision=B.SVT_FP64, oversample=10, power=2):
    return solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta, eps=eps, maxiter=maxiter,
                 incr=p.incr, precision=precision, svd_method=B.SVT_SVD_RANDOMIZED, rsvd_oversample=oversample,
                 rsvd_power=power, seed=SEED)


@pytest.mark.parametrize("power", [1, 3])
@pytest.mark.parametrize("case", [(400, 400, 10, 47400, 0), (157, 93, 4, 5200, 1)])
def test_fp64_matches_randomized_oracle(case, power):
    gpu_case(f"randomised SVD FP64 {case} power {power}")
    p = workload.gaussian_lowrank(*case) if case[0] != 400 else workload.config(1)
    k = 30
    o = svt_randomized(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, 0.0, k, p.incr, power=power, seed=SEED)
    g = _gpu(p, k, 0.0, power=power)
    assert g["status"] == B.SVT_NOT_CONVERGED and g["info"]["iters"] == o["iters"] == k
    assert g["info"]["k0"] == o["k0"]
    assert list(g["ranks"]) == o["ranks"] and list(g["s_hist"]) == o["s_hist"]
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=1e-8)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 1e-8


def test_full_width_is_exact():
    gpu_case("randomised SVD with full-width test matrices vs tier A")
    p = workload.gaussian_lowrank(120, 100, 3, 4000, 0, maxiter=300)
    o = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr)
    g = _gpu(p, p.maxiter, p.eps, oversample=1000, power=0)
    assert g["status"] == B.SVT_OK and o["status"] == "ok"
    assert g["info"]["iters"] == o["iters"] and list(g["ranks"]) == o["ranks"]
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=1e-8)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 1e-8


def test_mixed_matches_randomized_oracle():
    gpu_case("randomised SVD mixed 400^2")
    p = workload.config(1)
    k = 30
    o = svt_randomized(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, 0.0, k, p.incr, power=2, seed=SEED)
    g = _gpu(p, k, 0.0, precision=B.SVT_MIXED, power=2)
    assert g["info"]["iters"] == k
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=5e-4)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 5e-4


def test_refused_for_the_dantzig_selector():
    p = workload.gaussian_lowrank(60, 50, 2, 1500, 0)
    with pytest.raises(B.SvtError):
        solve(p.m, p.n, p.rows, p.cols, p.vals, svd_method=B.SVT_SVD_RANDOMIZED,
              constraint=B.SVT_CONSTRAINT_INEQUALITY, ineq_tol=0.1)


def test_step_cap_bounds_s():
    # lanczos_maxsteps caps s_k: a rank above it ends with SVT_ELANCZOS.  No
    # kick, so that the cap meets the randomised SVD, not the kick's
    # bidiagonalisation
    gpu_case("randomised SVD step cap")
    p = workload.config(1)
    with pytest.raises(B.SvtError) as e:
        _gpu_capped(p, 4, 20)
    assert e.value.status == B.SVT_ELANCZOS and "randomised" in str(e.value)
    assert e.value.info.iters >= 1
    g = _gpu_capped(p, 16, 5)
    assert g[0] == B.SVT_NOT_CONVERGED and g[1].iters == 5


def _gpu_capped(p, cap, maxiter):
    prm = B.svt_params_default(p.m, p.n, p.nnz)
    prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, p.delta, 0.0, maxiter, p.incr
    prm.kick = 0
    prm.svd_method = B.SVT_SVD_RANDOMIZED
    prm.seed = SEED
    prm.lanczos_maxsteps = cap
    h = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
    try:
        return B.svt_solve(h)
    finally:
        B.svt_destroy(h)
