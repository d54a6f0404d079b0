"""General linear operators (Section 3.1, eq. (3.3)) on the GPU against the
CPU oracle (needs an MI355X): the kick, the sampling operator written as a
general operator (the completion solve's result), and sparse random
measurements at a fixed iteration (FP64: same ranks, X within 1e-8; mixed
5e-4) and to convergence."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workload
from oracle.general import adjoint, svt_general
from paper_0810_3286_amd import solve
from paper_0810_3286_amd import svt as B
from tests.helpers import gpu_case, rel_diff_factored

pytestmark = pytest.mark.gpu


def _run(q, precision, eps, maxiter, delta=None, kick=1):
    prm = B.svt_params_default(q.m, q.n, q.p)
    prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = q.tau, delta or q.delta, eps, maxiter, q.incr
    prm.precision = precision
    prm.kick = kick
    h = B.svt_create_sensing(q.m, q.n, q.srows, q.scols, q.gptr, q.gidx, q.gval, q.b, prm)
    try:
        st, info = B.svt_solve(h)
        U, w, V = B.svt_factors(h, q.m, q.n)
        hist = B.svt_history(h)
    finally:
        B.svt_destroy(h)
    return st, info, U, V, hist


SENSE = [(80, 60, 3, 5, 3, 1), (61, 90, 2, 6, 4, 2), (150, 120, 4, 5, 3, 3)]


def _problem(c):
    m, n, r, f, cc, seed = c
    return workload.sparse_sensing(m, n, r, int(f * r * (m + n - r)), cc, seed=seed)


@pytest.mark.parametrize("case", SENSE)
def test_sensing_kick(case):
    gpu_case(f"sensing kick {case}")
    q = _problem(case)
    prm = B.svt_params_default(q.m, q.n, q.p)
    prm.tau, prm.delta = q.tau, q.delta
    h = B.svt_create_sensing(q.m, q.n, q.srows, q.scols, q.gptr, q.gidx, q.gval, q.b, prm)
    try:
        s1, k0 = B.svt_kick(h)
    finally:
        B.svt_destroy(h)
    so = oracle.jacobi_svd(adjoint(q.m, q.n, q.srows, q.scols, q.G(), q.b))[1][0]
    assert abs(s1 - so) <= 1e-11 * so
    assert k0 == oracle.k0_kick(q.tau, q.delta, so)


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
@pytest.mark.parametrize("case", SENSE)
def test_sensing_fixed_iteration_matches_oracle(case, precision):
    gpu_case(f"sensing 100 iterations {case} precision {precision}")
    q = _problem(case)
    o = svt_general(q.m, q.n, q.srows, q.scols, q.G(), q.b, q.tau, q.delta, 0.0, 100, q.incr)
    st, info, U, V, hist = _run(q, precision, 0.0, 100)
    assert st == B.SVT_NOT_CONVERGED and info.iters == 100 and info.k0 == o["k0"]
    tol = 1e-8 if precision == B.SVT_FP64 else 5e-4
    if precision == B.SVT_FP64:
        assert list(hist["ranks"]) == o["ranks"]
    np.testing.assert_allclose(hist["residuals"], o["residuals"], rtol=tol)
    assert rel_diff_factored(U, V, o["U"], o["V"]) <= tol


def test_sensing_converged_run_matches_oracle():
    gpu_case("sensing converged run")
    q = workload.sparse_sensing(80, 60, 3, 8 * 3 * 137, 3, seed=4)
    o = svt_general(q.m, q.n, q.srows, q.scols, q.G(), q.b, q.tau, q.delta, q.eps, 500, q.incr)
    assert o["status"] == "ok"
    st, info, U, V, hist = _run(q, B.SVT_FP64, q.eps, 500)
    assert st == B.SVT_OK and info.iters == o["iters"] and list(hist["ranks"]) == o["ranks"]
    assert rel_diff_factored(U, V, o["U"], o["V"]) <= 1e-8
    assert rel_diff_factored(U, V, q.ML, q.MR) <= 1e-2


def test_sampling_operator_as_general_operator():
    # G = identity on S = Omega: the completion solve's result, bit for bit
    # in iterations and ranks, X within 1e-12
    gpu_case("sampling operator through the general-operator entry point")
    p = workload.gaussian_lowrank(150, 120, 4, 7000, 6, maxiter=400)
    q = workload.SensingProblem(m=p.m, n=p.n, r=p.r, srows=p.rows, scols=p.cols,
                                gptr=np.arange(p.nnz + 1, dtype=np.int64), gidx=np.arange(p.nnz, dtype=np.int32),
                                gval=np.ones(p.nnz), b=p.vals, ML=p.ML, MR=p.MR, tau=p.tau, delta=p.delta,
                                eps=p.eps, maxiter=400, incr=p.incr)
    st, info, U, V, hist = _run(q, B.SVT_FP64, p.eps, 400)
    g = solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta, eps=p.eps, maxiter=400, incr=p.incr)
    assert info.iters == g["info"]["iters"] and list(hist["ranks"]) == list(g["ranks"])
    assert rel_diff_factored(U, V, g["U"], g["V"]) <= 1e-12
