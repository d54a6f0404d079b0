"""Full-size workloads on the GPU (needs an MI355X).

* 5000 x 5000, rank 10, |Omega| = 5 d_r against the stored tier-B oracle
  runs: at a fixed iteration (60) FP64 with the same ranks and X within
  1e-8, mixed within 5e-4; the complete runs by their shared history, their
  distance to the oracle's result and to the truth;
* 10000 x 10000, rank 50, |Omega| = 4 d_r against the stored tier-B X at
  iteration 40 (FP64 within 1e-8, mixed within 5e-4) and the stored tier-C
  complete run (FP64: same iterations and ranks, X within 1e-8, under both
  rank-decision rules; mixed: +-2 iterations, 5e-4);
* 30000 x 30000, rank 10, |Omega| = 6 d_r (the bench's workload, Table 1's
  last row) against the stored tier-C oracle run (Algorithm 1 with a library
  partial SVD): X^20, X^60 and the complete run, FP64 with the same
  iteration count and ranks, residual histories and X within 1e-8; mixed
  within +-2 iterations and 5e-4; and the rank decision of the
  bidiagonalisation with and without its certified early exit;
* 10000 x 10000 (rank 50) and 30000 x 30000 (rank 10) in the configuration
  the bench times, by properties that hold at any size: the reported residual
  equals the one recomputed in FP64 from the returned factors, the final rank
  is the truth's, the error against the truth is of the order of eps
  (Table 1), and the mixed and FP64 solves agree within 5e-4."""
import os

import numpy as np
import pytest

import oracle
import workload
from paper_0810_3286_amd import solve
from paper_0810_3286_amd import svt as B
from tests.helpers import gpu_case, rel_diff_factored

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _solve(p, precision):
    return solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta, eps=p.eps,
                 maxiter=p.maxiter, incr=p.incr, precision=precision)


def _gold(cfg):
    g = np.load(os.path.join(GOLDEN, f"oracle_config{cfg}.npz"))
    return dict(iters=int(g["iters"]), k0=int(g["k0"]), ranks=[int(x) for x in g["ranks"]],
                residuals=g["residuals"], U=g["U"], V=g["V"])


def _recomputed_residual(p, U, V):
    e = p.vals - oracle.sampled_entries(U, V, p.rows, p.cols)
    return float(np.linalg.norm(e) / np.linalg.norm(p.vals))


def _solve_fixed(p, precision, k):
    return solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta, eps=0.0,
                 maxiter=k, incr=p.incr, precision=precision)


# Near the end of the 5000^2 run sigma_11 and sigma_12 of the iterate hover
# around tau, the rank flips between 10, 11 and 12, and a rounding-level
# difference grows by orders of magnitude: between oracle runs that differ
# only by rounding, 1e-14 up to iteration 50, 8e-7 at 100, order one after
# 150 (tests/test_oracle_spread.py).  Exact parity is therefore checked at a
# fixed iteration (60), and the complete runs by what the oracle's own
# spread allows.
def test_5000_fp64_matches_stored_oracle_at_iteration_60():
    gpu_case("5000^2 rank 10 FP64, 60 iterations vs stored tier-B oracle")
    p = workload.config(2)
    o = _gold("2_k60")
    g = _solve_fixed(p, B.SVT_FP64, 60)
    assert g["status"] == B.SVT_NOT_CONVERGED and g["info"]["iters"] == 60 == o["iters"]
    assert g["info"]["k0"] == o["k0"]
    assert list(g["ranks"]) == o["ranks"]
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=1e-8)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 1e-8


def test_5000_mixed_matches_stored_oracle_at_iteration_60():
    gpu_case("5000^2 rank 10 mixed, 60 iterations vs stored tier-B oracle")
    p = workload.config(2)
    o = _gold("2_k60")
    g = _solve_fixed(p, B.SVT_MIXED, 60)
    assert list(g["ranks"]) == o["ranks"]
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=5e-4)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 5e-4


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
def test_5000_complete_run_against_stored_oracle(precision):
    gpu_case(f"5000^2 rank 10 precision {precision}, complete run vs stored tier-B oracle")
    p = workload.config(2)
    o = _gold(2)
    g = _solve(p, precision)
    assert g["status"] == B.SVT_OK and g["info"]["k0"] == o["k0"]
    # the trajectories agree until the amplified rounding reaches 1e-8 (FP64)
    head = 70 if precision == B.SVT_FP64 else 1
    tol = 1e-8 if precision == B.SVT_FP64 else 5e-4
    np.testing.assert_allclose(g["residuals"][:head], o["residuals"][:head], rtol=tol)
    assert list(g["ranks"][:60]) == o["ranks"][:60]
    # The oracle's own complete runs, with inputs or start vectors that
    # differ only by rounding, stop anywhere in a range of iterations and end
    # a few 1e-5 apart (tests/test_oracle_spread.py); the window and the
    # tolerance come from that spread, not from GPU runs
    from tests.test_oracle_spread import gpu_window
    lo, hi, xtol = gpu_window()
    assert lo <= g["info"]["iters"] <= hi
    tol_x = xtol if precision == B.SVT_FP64 else max(xtol, 5e-4)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= tol_x
    assert rel_diff_factored(g["U"], g["V"], p.ML, p.MR) < 2e-4


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
def test_10000_rank50_matches_stored_oracle_at_iteration_40(precision):
    # 10000 x 10000, rank 50, |Omega| = 4 d_r: the oracle's X at iteration 40
    # (eps = 0), stored; FP64 to 1e-8 with the same ranks, mixed to 5e-4
    gpu_case(f"10000^2 rank 50 precision {precision}, 40 iterations vs stored tier-B oracle")
    p = workload.config(3)
    o = _gold("3_k40")
    g = _solve_fixed(p, precision, 40)
    assert g["status"] == B.SVT_NOT_CONVERGED and g["info"]["iters"] == 40 == o["iters"]
    assert g["info"]["k0"] == o["k0"]
    assert list(g["ranks"]) == o["ranks"]
    tol = 1e-8 if precision == B.SVT_FP64 else 5e-4
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=tol)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= tol


@pytest.mark.parametrize("cfg,precision", [(3, B.SVT_MIXED), (4, B.SVT_MIXED), (4, B.SVT_FP64)])
def test_full_size_properties(cfg, precision):
    gpu_case(f"config {cfg} precision {precision}: full-size properties")
    p = workload.config(cfg)
    g = _solve(p, precision)
    assert g["status"] == B.SVT_OK
    # the truth's r components carry X: at 10000^2, rank 50, |Omega| = 4 d_r
    # a few singular values end just above tau (rank 58, weights below 1
    # against ~9000), in the FP64 and mixed runs alike
    r = g["info"]["rank"]
    w = np.asarray(g["w"])
    assert r >= p.r and np.all(w[p.r:] < 1e-3 * w[p.r - 1])
    # Table 1 and Section 5.2.1: fewer than 200 iterations at these sizes
    assert 80 <= g["info"]["iters"] < 200
    res = _recomputed_residual(p, g["U"], g["V"])
    # the FP32 sampled product perturbs x by ~1e-7 |x|, i.e. the residual
    # (~1e-4 ||P_Omega M||) by up to ~1e-3 of itself
    tol = 1e-8 if precision == B.SVT_FP64 else 1e-2
    assert abs(res - g["info"]["rel_residual"]) <= tol * res
    assert res <= p.eps * (1 + tol)
    # error against the truth of the order of the residual (Table 1: 1.6e-4
    # to 1.8e-4 at eps = 1e-4)
    assert rel_diff_factored(g["U"], g["V"], p.ML, p.MR) < 3e-4


def test_30000_mixed_agrees_with_fp64():
    gpu_case("30000^2 rank 10: mixed vs FP64")
    p = workload.config(4)
    g64 = _solve(p, B.SVT_FP64)
    g32 = _solve(p, B.SVT_MIXED)
    assert abs(g64["info"]["iters"] - g32["info"]["iters"]) <= 2
    n = min(len(g64["ranks"]), len(g32["ranks"]))
    assert list(g64["ranks"][:n]) == list(g32["ranks"][:n])
    assert rel_diff_factored(g32["U"], g32["V"], g64["U"], g64["V"]) <= 5e-4


# 30000 x 30000, rank 10: the stored tier-C oracle run (123 iterations, k0 4)
@pytest.mark.parametrize("k", [20, 60])
def test_30000_fp64_matches_stored_oracle_at_fixed_iteration(k):
    gpu_case(f"30000^2 rank 10 FP64, {k} iterations vs stored tier-C oracle")
    p = workload.config(4)
    o = _gold(f"4_k{k}")
    g = _solve_fixed(p, B.SVT_FP64, k)
    assert g["status"] == B.SVT_NOT_CONVERGED and g["info"]["iters"] == k == o["iters"]
    assert g["info"]["k0"] == o["k0"]
    assert list(g["ranks"]) == o["ranks"]
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=1e-8)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 1e-8


@pytest.mark.parametrize("margin", [0.05, 1.0])
def test_30000_fp64_complete_run_matches_stored_oracle(margin):
    # margin 0.05 (default): the rank decision may accept a Ritz value below
    # tau by its residual interval; margin 1.0: only converged values decide,
    # as Algorithm 1 does.  Both must give the oracle's rank sequence.
    gpu_case(f"30000^2 rank 10 FP64 complete run (decide_margin {margin}) vs stored tier-C oracle")
    p = workload.config(4)
    o = _gold(4)
    g = solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta, eps=p.eps,
              maxiter=p.maxiter, incr=p.incr, precision=B.SVT_FP64, decide_margin=margin)
    assert g["status"] == B.SVT_OK
    assert g["info"]["iters"] == o["iters"] and g["info"]["k0"] == o["k0"]
    assert list(g["ranks"]) == o["ranks"]
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=1e-8)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 1e-8


def test_30000_mixed_complete_run_against_stored_oracle():
    gpu_case("30000^2 rank 10 mixed complete run vs stored tier-C oracle")
    p = workload.config(4)
    o = _gold(4)
    g = _solve(p, B.SVT_MIXED)
    assert g["status"] == B.SVT_OK and g["info"]["k0"] == o["k0"]
    assert abs(g["info"]["iters"] - o["iters"]) <= 2
    n = min(len(g["ranks"]), len(o["ranks"]))
    assert list(g["ranks"][:n]) == o["ranks"][:n]
    np.testing.assert_allclose(g["residuals"][:n], o["residuals"][:n], rtol=5e-4)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 5e-4


# 10000 x 10000, rank 50, |Omega| = 4 d_r: the stored tier-C complete run
# (135 iterations, k0 4; the rank climbs from 50 to 58 from iteration 54 on,
# a few singular values ending just above tau)
@pytest.mark.parametrize("margin", [0.05, 1.0])
def test_10000_rank50_fp64_complete_run_matches_stored_oracle(margin):
    gpu_case(f"10000^2 rank 50 FP64 complete run (decide_margin {margin}) vs stored tier-C oracle")
    p = workload.config(3)
    o = _gold(3)
    g = solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta, eps=p.eps,
              maxiter=p.maxiter, incr=p.incr, precision=B.SVT_FP64, decide_margin=margin)
    assert g["status"] == B.SVT_OK
    assert g["info"]["iters"] == o["iters"] and g["info"]["k0"] == o["k0"]
    assert list(g["ranks"]) == o["ranks"]
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=1e-8)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 1e-8


def test_10000_rank50_mixed_complete_run_against_stored_oracle():
    gpu_case("10000^2 rank 50 mixed complete run vs stored tier-C oracle")
    p = workload.config(3)
    o = _gold(3)
    g = _solve(p, B.SVT_MIXED)
    assert g["status"] == B.SVT_OK and g["info"]["k0"] == o["k0"]
    assert abs(g["info"]["iters"] - o["iters"]) <= 2
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 5e-4
    # the rank sequence may differ where a value sits within the mixed
    # form's tie band of tau (1e-5 tau); the final ranks agree within one
    assert abs(int(g["ranks"][-1]) - o["ranks"][-1]) <= 1
