"""Tier C of the oracle (sparse iterate, the s_k largest triplets from a
library partial SVD) pinned to tiers A and B, which it shares no code with:

* tier A (dense Jacobi SVD of the dense iterate) on square, tall and wide
  problems and on the stored 400 x 400 run: the same iterations, ranks and
  s_k, residual histories within 1e-10 and X within 1e-10;
* tier B (Gram-matrix eigendecomposition) on the stored 5000 x 5000 run at
  iteration 60 (X within 1e-10), and, through the comparison that the
  goldens script stores, at 10000 x 10000, rank 50, iteration 40;
* the partial SVD step itself against LAPACK's full SVD of the dense matrix.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workload
from oracle.krylov import svt_krylov, top_triplets_sparse
from tests.helpers import rel_diff_factored

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("case", [(150, 150, 4, 7000, 6), (90, 260, 3, 8000, 3), (260, 90, 3, 8000, 5)])
def test_tier_c_matches_tier_a(case):
    p = workload.gaussian_lowrank(*case, maxiter=300)
    a = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr)
    c = svt_krylov(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr)
    assert (a["iters"], a["k0"], a["status"]) == (c["iters"], c["k0"], c["status"])
    assert a["ranks"] == c["ranks"] and a["s_hist"] == c["s_hist"]
    np.testing.assert_allclose(c["residuals"], a["residuals"], rtol=1e-10)
    assert rel_diff_factored(c["U"], c["V"], a["U"], a["V"]) <= 1e-10


def test_tier_c_matches_stored_tier_a_400():
    g = np.load(os.path.join(GOLDEN, "oracle_config1.npz"))
    p = workload.config(1)
    c = svt_krylov(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr)
    assert c["iters"] == int(g["iters"]) and c["ranks"] == list(g["ranks"])
    assert c["s_hist"] == list(g["s_hist"])
    np.testing.assert_allclose(c["residuals"], g["residuals"], rtol=1e-10)
    assert rel_diff_factored(c["U"], c["V"], g["U"], g["V"]) <= 1e-10


@pytest.mark.slow
def test_tier_c_matches_stored_tier_b_5000_k60():
    g = np.load(os.path.join(GOLDEN, "oracle_config2_k60.npz"))
    assert str(g["tier"]) == "B"
    p = workload.config(2)
    c = svt_krylov(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, 0.0, 60, p.incr)
    assert c["ranks"] == list(g["ranks"]) and c["s_hist"] == list(g["s_hist"])
    np.testing.assert_allclose(c["residuals"], g["residuals"], rtol=1e-10)
    assert rel_diff_factored(c["U"], c["V"], g["U"], g["V"]) <= 1e-10


def test_tier_c_matches_tier_b_10000_rank50_k40_stored_comparison():
    path = os.path.join(GOLDEN, "oracle_config3.npz")
    if not os.path.exists(path):
        pytest.skip("the 10000 x 10000 tier-C run is not stored")
    g = np.load(path)
    assert str(g["tier"]) == "C" and int(g["cross_k"]) == 40 and str(g["cross_tier"]) == "B"
    assert bool(g["cross_ranks_equal"]) and bool(g["cross_s_equal"])
    assert float(g["cross_res_rel_diff"]) <= 1e-10
    assert float(g["cross_x_rel_diff"]) <= 1e-10


@pytest.mark.parametrize("shape,s", [((60, 45), 5), ((45, 60), 7), ((120, 80), 1)])
def test_partial_svd_step_against_lapack(shape, s):
    rng = np.random.default_rng(11)
    A = sp.random(*shape, density=0.3, random_state=rng, data_rvs=rng.standard_normal).tocsr()
    U, S, V = top_triplets_sparse(A, s, seed=3)
    ref = np.linalg.svd(A.toarray(), compute_uv=False)
    np.testing.assert_allclose(S, ref[:s], rtol=1e-12)
    assert np.all(np.diff(S) <= 0)
    top = ref[0]
    assert np.linalg.norm(A @ V - U * S) <= 1e-12 * top
    assert np.linalg.norm(A.T @ U - V * S) <= 1e-12 * top
    np.testing.assert_allclose(U.T @ U, np.eye(s), atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(s), atol=1e-12)


def test_partial_svd_step_count_reaches_the_dimension():
    # s at min(m, n): the dense route (Jacobi) takes over and agrees with LAPACK
    rng = np.random.default_rng(5)
    A = sp.random(12, 9, density=0.6, random_state=rng, data_rvs=rng.standard_normal).tocsr()
    U, S, V = top_triplets_sparse(A, 9)
    np.testing.assert_allclose(S, np.linalg.svd(A.toarray(), compute_uv=False), rtol=1e-12, atol=1e-13)
    assert np.linalg.norm(A @ V - U * S) <= 1e-12 * S[0]


def test_stored_30000_run_is_consistent():
    """The stored 30000 x 30000 tier-C run: its X^20 and X^60 are prefixes of
    the complete run's history, the rank sequence is non-decreasing and ends
    at the truth's rank (Section 5.2.1), and the stop test holds exactly at
    the last iteration."""
    path = os.path.join(GOLDEN, "oracle_config4.npz")
    if not os.path.exists(path):
        pytest.skip("the 30000 x 30000 tier-C run is not stored")
    g = np.load(path)
    assert str(g["tier"]) == "C"
    ranks = list(g["ranks"])
    res = np.array(g["residuals"])
    assert int(g["iters"]) == len(ranks) and ranks[-1] == 10
    assert all(a <= b for a, b in zip(ranks, ranks[1:]))
    assert res[-1] <= 1e-4 < res[-2]
    for kk in (20, 60):
        s = np.load(os.path.join(GOLDEN, f"oracle_config4_k{kk}.npz"))
        assert int(s["iters"]) == kk
        assert list(s["ranks"]) == ranks[:kk]
        np.testing.assert_array_equal(s["residuals"], res[:kk])
