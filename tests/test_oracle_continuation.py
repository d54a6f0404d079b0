"""tau continuation with warm starts (Section 6) in the oracle, pinned by
what it must reduce to:

* a warm start from the kick's iterate k0 delta P_Omega(M) is the kicked run
  itself (eq. (5.3)): the y0 path and the kick path agree;
* a one-stage schedule is Algorithm 1;
* a warm-started stage ends, like a cold run at the same tau, within the
  stop tolerance of the same minimiser X*_tau, and in fewer iterations.
"""
import numpy as np

import oracle
import workload
from tests.helpers import rel_diff_factored


def _p():
    return workload.gaussian_lowrank(150, 120, 4, 7000, 6, maxiter=400)


def test_warm_start_from_the_kick_state_is_the_kicked_run():
    p = _p()
    a = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr)
    y0 = a["k0"] * p.delta * p.vals
    b = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr, y0=y0)
    assert b["iters"] == a["iters"] and b["ranks"] == a["ranks"] and b["k0"] == 0
    np.testing.assert_allclose(b["residuals"], a["residuals"], rtol=1e-12)
    assert rel_diff_factored(b["U"], b["V"], a["U"], a["V"]) <= 1e-12


def test_one_stage_schedule_is_algorithm_1():
    p = _p()
    a = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr)
    c = oracle.svt_continuation(p.m, p.n, p.rows, p.cols, p.vals, [p.tau], p.delta, p.eps, p.maxiter, p.incr)
    assert len(c) == 1 and c[0]["iters"] == a["iters"] and c[0]["ranks"] == a["ranks"]
    assert rel_diff_factored(c[0]["U"], c[0]["V"], a["U"], a["V"]) <= 1e-14


def test_warm_stage_reaches_the_cold_runs_minimiser():
    p = _p()
    s = np.sqrt(p.m * p.n)
    taus = [2.0 * s, 3.5 * s, 5.0 * s]
    stages = oracle.svt_continuation(p.m, p.n, p.rows, p.cols, p.vals, taus, p.delta, 1e-5, p.maxiter, p.incr)
    assert [st["status"] for st in stages] == ["ok"] * 3
    assert all(st["k0"] == 0 for st in stages[1:])
    cold = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, taus[-1], p.delta, 1e-5, p.maxiter, p.incr)
    # both end within the stop tolerance of the same minimiser
    assert rel_diff_factored(stages[-1]["U"], stages[-1]["V"], cold["U"], cold["V"]) <= 1e-4
    # the warm start is worth having: the last stage takes fewer iterations
    assert stages[-1]["iters"] < cold["iters"]
