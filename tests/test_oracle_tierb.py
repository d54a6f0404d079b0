"""Tier B of the oracle (sparse iterate, triplets from the Gram matrix) is
pinned to tier A (dense iterate, one-sided Jacobi) on sizes both can run:
the same iterations, ranks and s_k, residual histories within 1e-10 and the
same X within 1e-10; and its triplets are singular triplets of Y."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workload
from tests.helpers import rel_diff_factored


@pytest.mark.parametrize("case", [(150, 150, 4, 7000, 6), (90, 260, 3, 8000, 3), (260, 90, 3, 8000, 5)])
def test_tier_b_matches_tier_a(case):
    p = workload.gaussian_lowrank(*case, maxiter=300)
    a = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr)
    b = oracle.svt_sparse(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr)
    assert (a["iters"], a["k0"], a["status"]) == (b["iters"], b["k0"], b["status"])
    assert a["ranks"] == b["ranks"] and a["s_hist"] == b["s_hist"]
    np.testing.assert_allclose(b["residuals"], a["residuals"], rtol=1e-10)
    assert rel_diff_factored(b["U"], b["V"], a["U"], a["V"]) <= 1e-10


@pytest.mark.slow
def test_tier_b_matches_stored_tier_a_400():
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "oracle_config1.npz"))
    p = workload.config(1)
    b = oracle.svt_sparse(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr)
    assert b["iters"] == int(g["iters"]) and b["ranks"] == list(g["ranks"])
    assert rel_diff_factored(b["U"], b["V"], g["U"], g["V"]) <= 1e-10


def test_gram_triplets_are_singular_triplets():
    rng = np.random.default_rng(3)
    p = workload.gaussian_lowrank(120, 80, 3, 3000, 4)
    y = rng.standard_normal(p.nnz)
    Y = sp.csr_matrix((y, (p.rows, p.cols)), shape=(p.m, p.n))
    U, s, V, allsig = oracle.gram_triplets(Y, 2.0)
    ref = np.linalg.svd(Y.toarray(), compute_uv=False)
    np.testing.assert_allclose(allsig[:10], ref[:10], rtol=1e-12)
    assert s.shape[0] == int(np.count_nonzero(ref > 2.0))
    assert np.linalg.norm(Y @ V - U * s) <= 1e-11 * ref[0]
    assert np.linalg.norm(Y.T @ U - V * s) <= 1e-11 * ref[0]
