"""Pins for the oracle's Algorithm 1 (Section 5.1.5) and its building blocks.

* the kick (Section 5.1.3, eq. (5.3)): a run from Y^0 = 0 equals the kicked
  run shifted by k0, and X^k = 0, Y^k = k delta P_Omega(M) for k <= k0;
* full observation (Omega = every entry, delta = 1.2): every iterate keeps the
  singular vectors of M, so each singular value follows the scalar recursion
  y <- y + delta (sigma - (y - tau)_+) and the whole run (ranks, residuals,
  iteration count, X^opt) has a closed form;
* Theorem 4.2: for 0 < delta < 2, ||P_Omega(Y^k - Y*)||_F is non-increasing,
  and the limit satisfies the optimality conditions of eq. (2.8);
* exact recovery on a Gaussian low-rank instance (Table 1's regime): the
  relative error is of the order of eps (Section 5.1.4) and the rank sequence
  is non-decreasing (Section 2.2, Figure 1's observation);
* the sparse products and sampled entries against dense linear algebra.
"""
import math

import numpy as np
import pytest

import oracle
import workload


def _run(p, **kw):
    args = dict(tau=p.tau, delta=p.delta, eps=p.eps, maxiter=p.maxiter, incr=p.incr)
    args.update(kw)
    return oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, **args)


def test_k0_definition():
    # tau / (delta sigma1) in (k0 - 1, k0]
    assert oracle.k0_kick(10.0, 1.0, 5.0) == 2          # ratio exactly 2
    assert oracle.k0_kick(10.0, 1.0, 4.999) == 3        # ratio just above 2
    assert oracle.k0_kick(1.0, 2.0, 100.0) == 1         # ratio below 1
    for q in (0.3, 1.0, 2.5, 7.0, 7.000001):
        k0 = oracle.k0_kick(q, 1.0, 1.0)
        assert k0 - 1 < q <= k0


def test_kick_equals_unskipped_run_shifted():
    p = workload.gaussian_lowrank(40, 30, 3, 600, seed=5, maxiter=300)
    kicked = _run(p)
    plain = _run(p, kick=False, maxiter=300 + kicked["k0"])
    k0 = kicked["k0"]
    assert k0 >= 1
    # X^k = 0 for k <= k0 on the unskipped run
    assert plain["ranks"][:k0] == [0] * k0
    assert all(abs(r - 1.0) <= 1e-15 for r in plain["residuals"][:k0])
    # then it is the kicked run, shifted by k0
    assert plain["ranks"][k0:] == kicked["ranks"]
    assert plain["iters"] == kicked["iters"] + k0
    np.testing.assert_allclose(plain["residuals"][k0:], kicked["residuals"],
                               rtol=1e-9, atol=0)
    X1 = plain["U"] @ plain["V"].T
    X2 = kicked["U"] @ kicked["V"].T
    assert np.linalg.norm(X1 - X2) <= 1e-9 * np.linalg.norm(X2)


def test_kick_iterate_is_multiple_of_data():
    p = workload.gaussian_lowrank(25, 20, 2, 250, seed=6, maxiter=3)
    out = _run(p, kick=False, maxiter=12, keep_iterates=True)
    k0 = oracle.k0_kick(p.tau, p.delta, oracle.jacobi_svd(_dense_pm(p))[1][0])
    for k in range(1, k0 + 1):
        np.testing.assert_allclose(out["y_hist"][k], k * p.delta * p.vals, rtol=1e-14)


def _dense_pm(p):
    A = np.zeros((p.m, p.n))
    A[p.rows, p.cols] = p.vals
    return A


def full_observation_closed_form(sigma, tau, delta, eps, maxiter):
    """Scalar recursion for Omega = all entries (derived in the module doc)."""
    sigma = np.asarray(sigma, dtype=float)
    k0 = max(1, math.ceil(tau / (delta * sigma[0])))
    y = k0 * delta * sigma
    norm_m = math.sqrt(float(np.sum(sigma ** 2)))
    ranks, res = [], []
    for k in range(1, maxiter + 1):
        x = np.maximum(y - tau, 0.0)
        ranks.append(int(np.count_nonzero(y > tau)))
        res.append(math.sqrt(float(np.sum((sigma - x) ** 2))) / norm_m)
        if res[-1] <= eps:
            return dict(k0=k0, iters=k, ranks=ranks, residuals=res, x=x)
        y = y + delta * (sigma - x)
    return dict(k0=k0, iters=maxiter, ranks=ranks, residuals=res, x=x)


@pytest.mark.parametrize("m,n,sig", [
    (30, 20, [400.0, 150.0, 60.0, 20.0]),
    (16, 24, [300.0, 90.0, 45.0]),
    (12, 12, [500.0, 480.0, 30.0, 29.0, 5.3]),
    (30, 20, [90.0, 50.0, 21.0]),          # tau / (delta sigma_1) > 1: k0 = 2
])
def test_full_observation_closed_form(m, n, sig):
    sig = np.array(sig)
    p, U, s, V = workload.full_observation(m, n, sig, seed=m + n)
    out = _run(p)
    ref = full_observation_closed_form(sig, p.tau, p.delta, p.eps, p.maxiter)
    assert out["k0"] == ref["k0"]
    assert out["iters"] == ref["iters"]
    assert out["ranks"] == ref["ranks"]
    np.testing.assert_allclose(out["residuals"], ref["residuals"], rtol=1e-8, atol=1e-12)
    X = out["U"] @ out["V"].T
    Xref = (U * ref["x"]) @ V.T
    assert np.linalg.norm(X - Xref) <= 1e-10 * np.linalg.norm(Xref)


def test_theorem_4_2_monotone_dual_distance_and_limit():
    # delta < 2: ||P_Omega(Y^k - Y*)|| non-increasing; limit is optimal for (2.8)
    p = workload.gaussian_lowrank(8, 6, 1, 30, seed=5, delta=1.9)
    out = _run(p, eps=0.0, maxiter=4000, keep_iterates=True)
    ystar = out["y_hist"][-1]
    d = np.array([np.linalg.norm(y - ystar) for y in out["y_hist"]])
    assert d[-2] <= 1e-8 * d[0]                      # converged
    assert np.all(np.diff(d[:-50]) <= 1e-12 * d[0])  # non-increasing
    # KKT (eq. (5.4)): X* = D_tau(Y*) with P_Omega(X* - M) = 0 ...
    X = out["U"] @ out["V"].T
    assert np.abs(X[p.rows, p.cols] - p.vals).max() <= 1e-8 * np.abs(p.vals).max()
    # ... so X* minimises tau ||X||_* + 1/2 ||X||_F^2 over feasible X (eq. (2.8))
    rng = np.random.default_rng(0)
    mask = np.ones((p.m, p.n), dtype=bool)
    mask[p.rows, p.cols] = False

    def f(Z):
        return p.tau * np.linalg.svd(Z, compute_uv=False).sum() + 0.5 * np.linalg.norm(Z) ** 2

    f0 = f(X)
    for scale in (1e-1, 1e-3):
        for _ in range(20):
            D = rng.standard_normal((p.m, p.n)) * mask
            assert f(X + scale * D) >= f0 - 1e-9 * abs(f0)


@pytest.mark.slow
def test_exact_recovery_gaussian_low_rank():
    # Section 5.2.1 regime at a reduced size: n = 150, r = 5, |Omega| = 6 d_r.
    n, r = 150, 5
    nnz = 6 * workload.degrees_of_freedom(n, n, r)
    p = workload.gaussian_lowrank(n, n, r, nnz, seed=0, tau=5.0 * n)
    out = _run(p)
    assert out["status"] == "ok"
    assert 20 <= out["iters"] <= 200            # "fewer than 200 SVT iterations"
    ranks = out["ranks"]
    assert all(a <= b for a, b in zip(ranks, ranks[1:]))  # non-decreasing
    assert ranks[-1] == r
    X = out["U"] @ out["V"].T
    M = p.ML @ p.MR.T
    relerr = np.linalg.norm(X - M) / np.linalg.norm(M)
    # relative error of the order of the residual tolerance (Section 5.1.4)
    assert 1e-5 <= relerr <= 1e-3
    assert out["residuals"][-1] <= p.eps < out["residuals"][-2]


def test_sparse_products_match_dense():
    rng = np.random.default_rng(7)
    p = workload.gaussian_lowrank(37, 23, 2, 300, seed=8, shuffle=True)
    y = rng.standard_normal(p.nnz)
    Y = np.zeros((p.m, p.n))
    Y[p.rows, p.cols] = y
    x = rng.standard_normal(p.n)
    u = rng.standard_normal(p.m)
    np.testing.assert_allclose(oracle.apply_sparse(p.m, p.n, p.rows, p.cols, y, x),
                               Y @ x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oracle.apply_sparse(p.m, p.n, p.rows, p.cols, y, u, trans=True),
                               Y.T @ u, rtol=1e-13, atol=1e-13)
    U = rng.standard_normal((p.m, 4))
    V = rng.standard_normal((p.n, 4))
    np.testing.assert_allclose(oracle.sampled_entries(U, V, p.rows, p.cols),
                               (U @ V.T)[p.rows, p.cols], rtol=1e-13, atol=1e-13)
