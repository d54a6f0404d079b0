"""The stall bound (svt_params.stall_window) on the GPU.

Algorithm 1 stops only at its tolerance or at maxiter.  With the paper's step
1.2/p some requests of the serving stream oscillate without converging
(their rank and residual swing for hundreds of iterations); the stall bound
stops a run once `stall_window` consecutive iterations set no new minimum of
the recorded residual.  There is nothing in the paper to compare it with, so
these tests check the bound against its definition, applied here to the
residual history of the same run without it:

* a request that oscillates ends with SVT_STALLED at exactly the iteration
  the definition names, and its history is the unbounded run's, cut there;
* a converging run sets a new minimum at every iteration and is unchanged;
* the server applies the default window of 20 to a request that names none,
  and a negative window turns it off.
"""
import numpy as np
import pytest

import workload
from paper_0810_3286_amd import solve
from paper_0810_3286_amd import svt as B
from tests.helpers import gpu_case

pytestmark = pytest.mark.gpu


def _stall_iteration(res, window):
    """1-based iteration at which `window` consecutive iterations have set no
    new minimum of res, or None."""
    best, best_k = np.inf, 0
    for k, r in enumerate(res, start=1):
        if r < best:
            best, best_k = r, k
        elif k - best_k >= window:
            return k
    return None


def _oscillating_request():
    # request 20 of the serving stream (seed 0): 7035 x 610, rank 5,
    # |Omega| = 5.9 d_r; with delta = 1.2 / p its rank and residual oscillate
    spec = workload.serving_trace(32, seed=0, rate=1.0)[20][1]
    return workload.gaussian_lowrank(spec["m"], spec["n"], spec["r"], spec["nnz"], spec["seed"],
                                     noise_sigma=spec["noise_sigma"], maxiter=500)


def _kw(p, **kw):
    d = dict(tau=p.tau, delta=p.delta, eps=p.eps, incr=p.incr, precision=B.SVT_MIXED)
    d.update(kw)
    return d


@pytest.mark.parametrize("window", [10, 20])
def test_stall_bound_follows_its_definition(window):
    gpu_case(f"stall bound, oscillating request, window {window}")
    p = _oscillating_request()
    free = solve(p.m, p.n, p.rows, p.cols, p.vals, **_kw(p, maxiter=150))
    assert free["status"] == B.SVT_NOT_CONVERGED and free["info"]["iters"] == 150
    kt = _stall_iteration(free["residuals"], window)
    assert kt is not None and kt < 150
    cut = solve(p.m, p.n, p.rows, p.cols, p.vals, **_kw(p, maxiter=150, stall_window=window))
    assert cut["status"] == B.SVT_STALLED and cut["info"]["iters"] == kt
    assert list(cut["ranks"]) == list(free["ranks"][:kt])
    np.testing.assert_array_equal(cut["residuals"], free["residuals"][:kt])
    assert B.svt_status_string(B.SVT_STALLED).startswith("stalled")


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
def test_converging_run_is_unchanged(precision):
    gpu_case(f"stall bound, converging 400^2 run, precision {precision}")
    p = workload.config(1)
    kw = dict(tau=p.tau, delta=p.delta, eps=p.eps, maxiter=p.maxiter, incr=p.incr, precision=precision)
    a = solve(p.m, p.n, p.rows, p.cols, p.vals, **kw)
    b = solve(p.m, p.n, p.rows, p.cols, p.vals, stall_window=5, **kw)
    assert a["status"] == b["status"] == B.SVT_OK
    assert a["info"]["iters"] == b["info"]["iters"]
    assert np.all(np.diff(a["residuals"]) < 0)        # a new minimum every iteration
    np.testing.assert_array_equal(a["U"], b["U"])
    np.testing.assert_array_equal(a["V"], b["V"])


def test_server_default_window():
    gpu_case("stall bound, server default and opt-out")
    p = _oscillating_request()
    free = solve(p.m, p.n, p.rows, p.cols, p.vals, **_kw(p, maxiter=150))
    kt = _stall_iteration(free["residuals"], 20)
    srv = B.svt_server_create(8 << 30, 2)
    try:
        tickets = []
        for window in (0, -1):
            prm = B.svt_params_default(p.m, p.n, p.nnz)
            prm.tau, prm.delta, prm.eps, prm.incr, prm.maxiter = p.tau, p.delta, p.eps, p.incr, 150
            prm.precision = B.SVT_MIXED
            prm.stall_window = window
            prm.min_block_rows = 8      # the free run's row blocks: the same residuals
            tickets.append(B.svt_submit(srv, p.m, p.n, p.rows, p.cols, p.vals, prm))
        st0, info0 = B.svt_wait(srv, tickets[0])
        st1, info1 = B.svt_wait(srv, tickets[1])
        assert st0 == B.SVT_STALLED and info0.iters == kt
        assert st1 == B.SVT_NOT_CONVERGED and info1.iters == 150
        st, U, w, V, times = B.svt_result(srv, tickets[0], p.m, p.n)
        assert st == B.SVT_STALLED and U.shape[1] == info0.rank
    finally:
        B.svt_server_destroy(srv)
