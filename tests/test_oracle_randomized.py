"""The randomised-SVD oracle (Section 6's first direction) pinned on the CPU:

* the counter-based generator reproduces SplitMix64's published outputs
  (state 0 and the state after one step) and draws standard normals;
* with as many columns as the smaller dimension the range finder spans the
  whole space, so its triplets are the exact SVD (LAPACK);
* with enough power iterations the triplets converge to the exact ones;
* at a fixed small number of power iterations the SVT iteration does not
  reach eps = 1e-4 on the 400 x 400 workload, while the exact D_tau does in
  112 iterations: the approximate shrinkage leaves an error floor.
"""
import numpy as np
import scipy.sparse as sp

import oracle
import workload
from oracle.randomized import gaussian_matrix, randomized_triplets, splitmix_mix, svt_randomized
from tests.helpers import rel_diff_factored


def test_splitmix64_published_outputs():
    assert splitmix_mix(0) == 0xE220A8397B1DCDAF
    assert splitmix_mix(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4


def test_gaussian_draws():
    g = gaussian_matrix(2000, 500, 7, 3).ravel()
    n = g.shape[0]
    assert abs(g.mean()) <= 5.0 / np.sqrt(n)
    assert abs(g.var() - 1.0) <= 5.0 * np.sqrt(2.0 / n)
    assert not np.array_equal(gaussian_matrix(10, 3, 7, 3), gaussian_matrix(10, 3, 7, 4))
    np.testing.assert_array_equal(gaussian_matrix(10, 3, 7, 3), gaussian_matrix(10, 3, 7, 3))


def _sparse(m, n, seed):
    rng = np.random.default_rng(seed)
    return sp.random(m, n, density=0.3, random_state=rng, data_rvs=rng.standard_normal).tocsr()


def test_full_width_is_the_exact_svd():
    A = _sparse(60, 40, 1)
    U, S, V = randomized_triplets(A, 8, 100, 0, 0, 0)
    ref = np.linalg.svd(A.toarray(), compute_uv=False)
    np.testing.assert_allclose(S, ref[:8], rtol=1e-12)
    assert np.linalg.norm(A @ V - U * S) <= 1e-11 * ref[0]


def test_power_iterations_converge_to_the_exact_triplets():
    A = _sparse(120, 90, 2)
    ref = np.linalg.svd(A.toarray(), compute_uv=False)
    errs = [np.max(np.abs(randomized_triplets(A, 5, 5, q, 0, 0)[1] - ref[:5])) / ref[0] for q in (0, 4, 100)]
    assert errs[2] <= 1e-10 and errs[0] > errs[1] > errs[2]


def test_fixed_power_iterations_leave_an_error_floor():
    p = workload.config(1)
    r = svt_randomized(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, 200, p.incr, power=2)
    assert r["status"] == "not_converged" and min(r["residuals"]) > 10 * p.eps
    g = np.load(__import__("os").path.join(__import__("os").path.dirname(__file__), "golden", "oracle_config1.npz"))
    assert int(g["iters"]) == 112
    assert rel_diff_factored(r["U"], r["V"], p.ML, p.MR) > 0.01
