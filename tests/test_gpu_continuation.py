"""tau continuation with warm starts (Section 6) on the GPU against the CPU
oracle (needs an MI355X): svt_solve_path over a tau schedule, stage by stage
(FP64: the same iterations and ranks, X within 1e-8; mixed: +-2 iterations,
5e-4), and a warm start from the kick's iterate, set through the C ABI,
against the kicked solve."""
import numpy as np
import pytest

import oracle
import workload
from paper_0810_3286_amd import svt as B
from tests.helpers import gpu_case, rel_diff_factored

pytestmark = pytest.mark.gpu

CASES = [(150, 120, 4, 7000, 6), (90, 260, 3, 8000, 3)]


def _handle(p, precision, eps):
    prm = B.svt_params_default(p.m, p.n, p.nnz)
    prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, p.delta, eps, 400, p.incr
    prm.precision = precision
    return B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
@pytest.mark.parametrize("case", CASES)
def test_solve_path_matches_oracle(case, precision):
    gpu_case(f"tau continuation {case} precision {precision}")
    p = workload.gaussian_lowrank(*case, maxiter=400)
    s = np.sqrt(p.m * p.n)
    taus = [2.0 * s, 3.5 * s, 5.0 * s]
    eps = 1e-5
    o = oracle.svt_continuation(p.m, p.n, p.rows, p.cols, p.vals, taus, p.delta, eps, 400, p.incr)
    h = _handle(p, precision, eps)
    try:
        st, infos = B.svt_solve_path(h, taus)
        U, w, V = B.svt_factors(h, p.m, p.n)
        hist = B.svt_history(h)
    finally:
        B.svt_destroy(h)
    assert st == B.SVT_OK and len(infos) == 3
    assert [i.k0 for i in infos][1:] == [0, 0] and infos[0].k0 == o[0]["k0"]
    if precision == B.SVT_FP64:
        assert [i.iters for i in infos] == [x["iters"] for x in o]
        assert list(hist["ranks"]) == o[-1]["ranks"]
        np.testing.assert_allclose(hist["residuals"], o[-1]["residuals"], rtol=1e-8)
        assert rel_diff_factored(U, V, o[-1]["U"], o[-1]["V"]) <= 1e-8
    else:
        assert all(abs(i.iters - x["iters"]) <= 2 for i, x in zip(infos, o))
        assert rel_diff_factored(U, V, o[-1]["U"], o[-1]["V"]) <= 5e-4


def test_warm_start_from_the_kick_state_is_the_kicked_solve():
    gpu_case("warm start from k0 delta M")
    p = workload.gaussian_lowrank(*CASES[0], maxiter=400)
    h = _handle(p, B.SVT_FP64, p.eps)
    try:
        st, a = B.svt_solve(h)
        Ua, wa, Va = B.svt_factors(h, p.m, p.n)
        B.svt_set_iterate(h, a.k0 * p.delta * p.vals)
        prm = B.svt_params_default(p.m, p.n, p.nnz)
    finally:
        B.svt_destroy(h)
    prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, p.delta, p.eps, 400, p.incr
    prm.warm_start = 1
    h = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
    try:
        B.svt_set_iterate(h, a.k0 * p.delta * p.vals)
        st, b = B.svt_solve(h)
        Ub, wb, Vb = B.svt_factors(h, p.m, p.n)
    finally:
        B.svt_destroy(h)
    assert b.k0 == 0 and b.iters == a.iters
    assert rel_diff_factored(Ub, Vb, Ua, Va) <= 1e-12
