"""Serving form on the GPU: continuous batching of mixed-size requests.

* every result is bit-identical alone (svt_solve) and in the mix (server);
* admission respects the device-memory budget (a budget that fits one
  request at a time serialises the solves);
* a request solved in the mix matches the FP64 oracle (sampled subset).
The paper has no serving form: parity beyond alone = in the mix and the
oracle on sampled requests is unpinned."""
import numpy as np
import pytest

import oracle
import workload
from paper_0810_3286_amd import svt as B
from tests.helpers import gpu_case, rel_diff_factored

pytestmark = pytest.mark.gpu

REQS = [
    (150, 150, 4, 7000, 6),
    (90, 260, 3, 8000, 3),
    (260, 90, 3, 8000, 5),
    (400, 400, 10, 47400, 0),
    (700, 500, 5, 42000, 11),
    (33, 29, 2, 700, 3),
]


def _prm(p, precision):
    prm = B.svt_params_default(p.m, p.n, p.nnz)
    prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, p.delta, p.eps, 300, p.incr
    prm.precision = precision
    return prm


def _alone(p, prm):
    h = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
    try:
        st, info = B.svt_solve(h)
        U, w, V = B.svt_factors(h, p.m, p.n)
    finally:
        B.svt_destroy(h)
    return st, info, U, w, V


def _prm_alone(p, precision):
    # a request served with min_block_rows left 0 runs with the server's 64
    prm = _prm(p, precision)
    prm.min_block_rows = 64
    return prm


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
def test_alone_equals_mix(precision):
    gpu_case(f"serving alone vs mix precision {precision}")
    probs = [workload.gaussian_lowrank(*c, shuffle=True) for c in REQS]
    alone = [_alone(p, _prm_alone(p, precision)) for p in probs]
    srv = B.svt_server_create(64 << 30, 4)
    try:
        tickets = [B.svt_submit(srv, p.m, p.n, p.rows, p.cols, p.vals, _prm(p, precision)) for p in probs]
        for p, t, a in zip(probs, tickets, alone):
            st, info = B.svt_wait(srv, t)
            st2, U, w, V, times = B.svt_result(srv, t, p.m, p.n)
            assert st == a[0] and info.iters == a[1].iters
            assert np.array_equal(U, a[2]) and np.array_equal(w, a[3]) and np.array_equal(V, a[4])
            assert times[0] <= times[1] <= times[2]
        stats = B.svt_server_stats(srv)
        assert stats["max_running"] >= 2  # the solves overlapped
    finally:
        B.svt_server_destroy(srv)


def test_budget_serialises():
    gpu_case("serving tiny budget")
    probs = [workload.gaussian_lowrank(*c) for c in REQS[:4]]
    fps = [B.svt_footprint(p.m, p.n, p.nnz) for p in probs]
    budget = int(max(fps) * 1.01)
    srv = B.svt_server_create(budget, 4)
    try:
        tickets = [B.svt_submit(srv, p.m, p.n, p.rows, p.cols, p.vals, _prm(p, B.SVT_FP64)) for p in probs]
        spans = []
        for p, t in zip(probs, tickets):
            B.svt_wait(srv, t)
            spans.append(B.svt_result(srv, t, p.m, p.n)[4])
        stats = B.svt_server_stats(srv)
        assert stats["peak_bytes"] <= budget
        # a pair of requests fits only if both footprints fit
        for i in range(len(spans)):
            for j in range(i + 1, len(spans)):
                overlap = min(spans[i][2], spans[j][2]) > max(spans[i][1], spans[j][1])
                if fps[i] + fps[j] > budget:
                    assert not overlap
        # first come, first served
        starts = [s[1] for s in spans]
        assert starts == sorted(starts)
    finally:
        B.svt_server_destroy(srv)


def test_mix_member_matches_oracle():
    gpu_case("serving vs oracle")
    probs = [workload.gaussian_lowrank(*c) for c in REQS[:3]]
    srv = B.svt_server_create(64 << 30, 3)
    try:
        tickets = [B.svt_submit(srv, p.m, p.n, p.rows, p.cols, p.vals, _prm(p, B.SVT_FP64)) for p in probs]
        for p, t in zip(probs, tickets):
            st, info = B.svt_wait(srv, t)
            _, U, w, V, _ = B.svt_result(srv, t, p.m, p.n)
            o = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, 300, p.incr)
            assert info.iters == o["iters"]
            assert rel_diff_factored(U, V, o["U"], o["V"]) <= 1e-8
    finally:
        B.svt_server_destroy(srv)


def test_failing_request_frees_its_slot():
    # a request that hits its step cap ends with SVT_ELANCZOS and rank 0;
    # the request queued behind it on the single slot still completes
    gpu_case("serving: failing request then a normal one, one slot")
    hard = workload.gaussian_lowrank(700, 500, 5, 30000, 11, shuffle=True)
    easy = workload.gaussian_lowrank(*REQS[0], shuffle=True)
    prm_h = _prm(hard, B.SVT_MIXED)
    prm_h.maxiter, prm_h.lanczos_maxsteps = 60, 64
    srv = B.svt_server_create(64 << 30, 1)
    try:
        t1 = B.svt_submit(srv, hard.m, hard.n, hard.rows, hard.cols, hard.vals, prm_h)
        t2 = B.svt_submit(srv, easy.m, easy.n, easy.rows, easy.cols, easy.vals, _prm(easy, B.SVT_MIXED))
        st1, info1 = B.svt_wait(srv, t1)
        st1b, U, w, V, times1 = B.svt_result(srv, t1, hard.m, hard.n)
        st2, info2 = B.svt_wait(srv, t2)
        _, _, _, _, times2 = B.svt_result(srv, t2, easy.m, easy.n)
        B.svt_release(srv, t1)
        B.svt_release(srv, t2)
    finally:
        B.svt_server_destroy(srv)
    assert st1 == st1b == B.SVT_ELANCZOS and info1.iters >= 1 and U.shape == (hard.m, 0)
    assert st2 == B.SVT_OK
    assert times1[0] <= times1[1] <= times1[2] <= times2[1] <= times2[2]


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
def test_footprint_bounds_the_device_bytes(precision):
    # the admission footprint is an upper bound of what a handle run with the
    # served step cap (512) ever holds, basis growth included
    for c in [(700, 500, 5, 42000, 11), (2400, 1800, 50, 4 * 50 * (2400 + 1800 - 50), 2),
              (3000, 250, 10, 6 * 10 * (3250 - 10), 4)]:
        gpu_case(f"footprint vs device bytes {c} precision {precision}")
        p = workload.gaussian_lowrank(*c, maxiter=60)
        prm = _prm(p, precision)
        prm.maxiter = 60
        prm.lanczos_maxsteps = 512
        h = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
        try:
            try:
                B.svt_solve(h)
            except B.SvtError:
                pass  # the bound must hold whatever the outcome
            cur, peak = B.svt_device_bytes(h)
        finally:
            B.svt_destroy(h)
        fp = B.svt_footprint(p.m, p.n, p.nnz, precision)
        assert 0 < cur <= peak <= fp, (c, cur, peak, fp)


def test_serving_stream_members_match_stored_oracle():
    # four requests drawn by the serving stream's own generator (seed 0,
    # sizes 622 to 7506, ranks 10 and 20), submitted together and solved in
    # the mix in the served (mixed) precision, each stopped at iteration 30
    # and compared with the stored oracle X^30 at the mixed form's 5e-4
    import os
    gpu_case("serving stream members vs stored oracle at iteration 30")
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "oracle_serving_k30.npz"))
    k = int(g["k"])
    trace = workload.serving_trace(32, seed=0, rate=1.0)
    probs = []
    for i in g["requests"]:
        spec = trace[int(i)][1]
        probs.append((int(i), workload.gaussian_lowrank(spec["m"], spec["n"], spec["r"], spec["nnz"], spec["seed"],
                                                        noise_sigma=spec["noise_sigma"], maxiter=500)))
    srv = B.svt_server_create(64 << 30, 4)
    try:
        tickets = []
        for i, p in probs:
            prm = B.svt_params_default(p.m, p.n, p.nnz)
            prm.tau, prm.delta, prm.incr = p.tau, p.delta, p.incr
            prm.eps, prm.maxiter = 0.0, k
            prm.precision = B.SVT_MIXED
            prm.stall_window = -1       # a fixed iteration count: no stall bound
            tickets.append(B.svt_submit(srv, p.m, p.n, p.rows, p.cols, p.vals, prm))
        for (i, p), t in zip(probs, tickets):
            st, info = B.svt_wait(srv, t)
            st2, U, w, V, times = B.svt_result(srv, t, p.m, p.n)
            assert st == B.SVT_NOT_CONVERGED and info.iters == k and info.k0 == int(g[f"r{i}_k0"])
            assert info.rank == int(g[f"r{i}_ranks"][-1])
            assert rel_diff_factored(U, V, g[f"r{i}_U"], g[f"r{i}_V"]) <= 5e-4, i
        assert B.svt_server_stats(srv)["max_running"] >= 2
    finally:
        B.svt_server_destroy(srv)
