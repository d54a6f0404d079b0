"""The degrees-of-freedom bound (svt_params.dof_bound) on the GPU.

A rank-r matrix of size m x n has r (m + n - r) degrees of freedom (Section
1.1); with fewer observations than that no method can determine it.  With
dof_bound > 0 a solve stops (SVT_UNDERDETERMINED) at the first step whose
iterate would have a rank r with r (m + n - r) > dof_bound |Omega|, before
that step's update; the factors keep the last completed iterate.  The Ritz
values of the bidiagonalisation bound the singular values from below, so the
count of Ritz values above tau settles it at the step where the unbounded
run's rank first passes the largest rank allowed.  There is nothing in the
paper to compare the bound with, so these tests check it against its
definition, applied to the history of the same run without it:

* a run whose rank passes the largest rank allowed ends with
  SVT_UNDERDETERMINED after exactly the iterations the definition names,
  with the unbounded run's history cut there and, bit for bit, the factors
  of the unbounded run stopped at that iteration;
* a run whose rank stays within the bound is unchanged bit for bit;
* the server applies dof_bound = 1 to a request that names none, and a
  negative value turns it off;
* with a general operator (Section 3.1) the observations counted are the
  measurements, not the support.
"""
import numpy as np
import pytest

import workload
from paper_0810_3286_amd import solve
from paper_0810_3286_amd import svt as B
from tests.helpers import gpu_case

pytestmark = pytest.mark.gpu


def _dof(r, m, n):
    return r * (m + n - r)


def _bound_for(rmax, p):
    """A dof_bound whose largest allowed rank is rmax: halfway between the
    degrees of freedom of rank rmax and rmax + 1, per observation."""
    return 0.5 * (_dof(rmax, p.m, p.n) + _dof(rmax + 1, p.m, p.n)) / p.nnz


def _kw(p, precision, **kw):
    d = dict(tau=p.tau, delta=p.delta, eps=p.eps, maxiter=p.maxiter, incr=p.incr, precision=precision)
    d.update(kw)
    return d


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
def test_bound_follows_its_definition(precision):
    gpu_case(f"dof bound, 400^2 run cut above its first rank, precision {precision}")
    p = workload.config(1)
    free = solve(p.m, p.n, p.rows, p.cols, p.vals, **_kw(p, precision))
    assert free["status"] == B.SVT_OK
    ranks = list(free["ranks"])
    rmax = ranks[0]
    assert max(ranks) > rmax
    # the definition: the first iteration whose rank passes rmax ends the run
    # before its update
    kt = next(i for i, r in enumerate(ranks) if r > rmax)
    assert kt >= 1
    cut = solve(p.m, p.n, p.rows, p.cols, p.vals, **_kw(p, precision, dof_bound=_bound_for(rmax, p)))
    assert cut["status"] == B.SVT_UNDERDETERMINED and cut["info"]["iters"] == kt
    assert list(cut["ranks"]) == ranks[:kt]
    np.testing.assert_array_equal(cut["residuals"], free["residuals"][:kt])
    # the factors are those of the last completed iterate
    stop = solve(p.m, p.n, p.rows, p.cols, p.vals, **_kw(p, precision, maxiter=kt, eps=0.0))
    assert stop["info"]["iters"] == kt and cut["info"]["rank"] == ranks[kt - 1]
    np.testing.assert_array_equal(cut["U"], stop["U"])
    np.testing.assert_array_equal(cut["V"], stop["V"])
    assert B.svt_status_string(B.SVT_UNDERDETERMINED).startswith("underdetermined")
    # below the first iterate's rank: no iteration completes, X stays 0
    none = solve(p.m, p.n, p.rows, p.cols, p.vals, **_kw(p, precision, dof_bound=_bound_for(rmax - 1, p)))
    assert none["status"] == B.SVT_UNDERDETERMINED and none["info"]["iters"] == 0
    assert none["info"]["rank"] == 0 and len(none["ranks"]) == 0 and none["U"].shape == (p.m, 0)


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
def test_run_within_the_bound_is_unchanged(precision):
    gpu_case(f"dof bound, converging 400^2 run within the bound, precision {precision}")
    p = workload.config(1)
    a = solve(p.m, p.n, p.rows, p.cols, p.vals, **_kw(p, precision))
    b = solve(p.m, p.n, p.rows, p.cols, p.vals, **_kw(p, precision, dof_bound=1.0))
    assert a["status"] == b["status"] == B.SVT_OK
    assert a["info"]["iters"] == b["info"]["iters"]
    assert _dof(max(a["ranks"]), p.m, p.n) <= p.nnz
    np.testing.assert_array_equal(a["U"], b["U"])
    np.testing.assert_array_equal(a["V"], b["V"])


def test_server_default_bound():
    # request 4 of the serving stream (seed 0): 1103 x 2748, rank 10, |Omega|
    # = 3.1 d_r; its iterate's rank swings past the largest rank its
    # observations allow (about 30), and without the bound it ends at the
    # stall bound instead
    gpu_case("dof bound, server default and opt-out")
    spec = workload.serving_trace(8, seed=0, rate=1.0)[4][1]
    p = workload.gaussian_lowrank(spec["m"], spec["n"], spec["r"], spec["nnz"], spec["seed"],
                                  noise_sigma=spec["noise_sigma"], maxiter=500)
    kw = _kw(p, B.SVT_MIXED, maxiter=150, lanczos_maxsteps=512, stall_window=20, min_block_rows=8)
    alone = {d: solve(p.m, p.n, p.rows, p.cols, p.vals, **kw, dof_bound=d) for d in (1.0, 0.0)}
    assert alone[1.0]["status"] == B.SVT_UNDERDETERMINED
    assert alone[0.0]["status"] != B.SVT_UNDERDETERMINED
    assert alone[1.0]["info"]["iters"] < alone[0.0]["info"]["iters"]
    srv = B.svt_server_create(8 << 30, 2)
    try:
        tickets = []
        for dof in (0.0, -1.0):
            prm = B.svt_params_default(p.m, p.n, p.nnz)
            prm.tau, prm.delta, prm.eps, prm.incr, prm.maxiter = p.tau, p.delta, p.eps, p.incr, 150
            prm.precision = B.SVT_MIXED
            prm.min_block_rows = 8      # the runs alone: the same row blocks
            prm.dof_bound = dof
            tickets.append(B.svt_submit(srv, p.m, p.n, p.rows, p.cols, p.vals, prm))
        for t, ref in zip(tickets, (alone[1.0], alone[0.0])):
            st, info = B.svt_wait(srv, t)
            assert st == ref["status"] and info.iters == ref["info"]["iters"]
            st, U, w, V, times = B.svt_result(srv, t, p.m, p.n)
            np.testing.assert_array_equal(U, ref["U"])
            np.testing.assert_array_equal(V, ref["V"])
    finally:
        B.svt_server_destroy(srv)


def _sensing(q, dof_bound):
    prm = B.svt_params_default(q.m, q.n, q.p)
    prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = q.tau, q.delta, q.eps, 500, q.incr
    prm.dof_bound = dof_bound
    h = B.svt_create_sensing(q.m, q.n, q.srows, q.scols, q.gptr, q.gidx, q.gval, q.b, prm)
    try:
        st, info = B.svt_solve(h)
        U, w, V = B.svt_factors(h, q.m, q.n)
        hist = B.svt_history(h)
    finally:
        B.svt_destroy(h)
    return st, info, U, V, hist


def test_general_operator_counts_measurements():
    # with a general operator (Section 3.1) the observations are the
    # measurements b, not the support: the bound's largest rank follows p
    gpu_case("dof bound, general operator")
    q = workload.sparse_sensing(150, 120, 4, int(5 * 4 * (150 + 120 - 4)), 3, seed=3)
    st, info, U, V, hist = _sensing(q, 0.0)
    assert st == B.SVT_OK
    ranks = list(hist["ranks"])
    dof = lambda r: r * (q.m + q.n - r)
    if max(ranks) > ranks[0]:
        rmax = ranks[0]
        kt = next(i for i, r in enumerate(ranks) if r > rmax)
        st2, info2, U2, V2, hist2 = _sensing(q, 0.5 * (dof(rmax) + dof(rmax + 1)) / q.p)
        assert st2 == B.SVT_UNDERDETERMINED and info2.iters == kt
        assert list(hist2["ranks"]) == ranks[:kt]
        np.testing.assert_array_equal(hist2["residuals"], hist["residuals"][:kt])
    # below the first iterate's rank, counted against the measurements: no
    # iteration completes
    r0 = ranks[0]
    st3, info3, U3, V3, hist3 = _sensing(q, 0.5 * (dof(r0 - 1) + dof(r0)) / q.p)
    assert st3 == B.SVT_UNDERDETERMINED and info3.iters == 0 and U3.shape == (q.m, 0)
    # (the same bound counted against the support instead would allow rank
    # r0, so the stop shows which count the library takes)
    if r0 >= 2:
        assert dof(r0) <= 0.5 * (dof(r0 - 1) + dof(r0)) / q.p * len(q.srows)
