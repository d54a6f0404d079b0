"""Partial reorthogonalisation of the bidiagonalisation (Section 5.1.1),
on the CPU.

The oracle (``oracle/partial_reorth.py``) is pinned to what the mathematics
fixes, not to itself:

* the two recurrences of the estimate are identities for the computed
  vectors: fed the actual inner products of one step, they give the actual
  inner products of the next to rounding, also long after orthogonality is
  lost (a dropped term or a wrong index fails this at O(1));
* the estimate bounds the loss it estimates, vector by vector;
* without reorthogonalisation the Ritz values repeat (ghosts), with full or
  partial reorthogonalisation they do not, and partial reorthogonalisation
  keeps the bases semi-orthogonal and reaches the full method's decision,
  steps and Ritz values while orthogonalising a minority of the vectors.

The library's host code for it (``orth_estimate.cpp``: the same estimate and
the schedule the solver uses, which decides each vector before its
coefficients reach the host) is compiled here with g++ and checked against
the oracle: its estimates equal the oracle's, and driving the oracle's
bidiagonalisation with its decisions, the coefficients arriving 2 to 10
steps late, keeps the bases semi-orthogonal with the full method's result
(FP64 and FP32 vectors), while a level above sqrt(u) is reported by its
check.  Nothing runs on a GPU.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import workload
from oracle import partial_reorth as pr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0810_3286_amd", "csrc")


def _dense_problem(m=300, n=200, r=8, noise=0.01, seed=1):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, r)) @ rng.standard_normal((r, n)) + noise * rng.standard_normal((m, n))


def _kick_iterate(idx):
    """The iterate Y^{k0} = k0 delta P_Omega M of a workload (eq. (5.3)),
    sparse, with the kick's k0 from ||P_Omega M||_2."""
    p = workload.config(idx)
    P = sp.csr_matrix((p.vals, (p.rows, p.cols)), shape=(p.m, p.n))
    s1 = sp.linalg.svds(P, k=1, return_singular_vectors=False)[0]
    k0 = int(np.ceil(p.tau / (p.delta * s1)))
    return (k0 * p.delta) * P, p.tau


_LATER = {}


def _later_iterate(idx, iters):
    """The iterate after `iters` SVT iterations of the tier-C oracle (the
    bidiagonalisations of later iterations run longer: 55 steps at 400^2,
    111 at 5000^2, where orthogonality is lost fast)."""
    key = (idx, iters)
    if key not in _LATER:
        from oracle import krylov
        p = workload.config(idx)
        o = krylov.svt_krylov(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, 0.0, iters, p.incr)
        _LATER[key] = (sp.csr_matrix((o["y_last"], (p.rows, p.cols)), shape=(p.m, p.n)), p.tau)
    return _LATER[key]


def _case(case):
    if case == "dense":
        return None
    if case == "later1":
        return _later_iterate(1, 5)
    if case == "later2":
        return _later_iterate(2, 3)
    return _kick_iterate(1 if case == "config1" else 2)


def _actual(run, k):
    U, V = run["U"][:, :k], run["V"][:, :k + 1]
    return U.T @ U, V.T @ V


def test_recurrences_are_identities_for_the_computed_vectors():
    A = _dense_problem()
    k = 80
    run = pr.gkl(A, k, policy="none")
    MU, NU = _actual(run, k)
    alpha, beta = run["alpha"], run["beta"]
    assert np.max(np.abs(MU - np.eye(k))) > 0.1      # orthogonality is long lost
    worst = 0.0
    for j in range(2, k + 1):                         # u_j, then v_{j+1}
        est = pr.OmegaEstimate(unit=0.0, dim=2)
        est.alpha = list(alpha[:j - 1])
        est.beta = list(beta[:j])                     # beta[i] = beta_{i+1}, beta[0] = 0
        est.mu = [MU[jj - 1, :jj - 1] for jj in range(1, j)]
        est.nu = [NU[jj - 1, :jj - 1] for jj in range(1, j + 1)]
        row = est.row_u(alpha[j - 1])
        worst = max(worst, np.max(np.abs(row - MU[j - 1, :j - 1])))
        est.push_u(alpha[j - 1], MU[j - 1, :j - 1], False)
        row = est.row_v(beta[j])
        worst = max(worst, np.max(np.abs(row - NU[j, :j])))
    assert worst < 1e-9


def test_estimate_bounds_the_loss():
    A = _dense_problem(seed=2)
    run = pr.gkl(A, 60, policy="none")
    for est, loss in ((run["est_u"], run["loss_u"]), (run["est_v"], run["loss_v"])):
        live = loss < 1e-3                              # before the loss saturates
        assert live.sum() > 10
        assert np.all(est[live] >= loss[live])


def _min_ratio(run):
    est = np.r_[run["est_u"][1:], run["est_v"]]
    loss = np.r_[run["loss_u"][1:], run["loss_v"]]
    live = (loss < 1e-3) & (loss > 0)                   # before the loss saturates
    return float(np.min(est[live] / loss[live])), int(live.sum())


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fp32_storage_estimate_bounds_the_loss(seed):
    # vectors stored in FP32 (the mixed form): the rounding term with c = 1
    ratio, n = _min_ratio(pr.gkl(_dense_problem(seed=seed), 60, policy="none", store="f32"))
    assert n > 10 and ratio >= 1.0


@pytest.mark.parametrize("case", ["config1", "later1"])
def test_fp32_storage_on_a_completion_iterate(case):
    Y, _ = _case(case)
    ratio, n = _min_ratio(pr.gkl(Y, 50, policy="none", store="f32"))
    assert n > 10 and ratio >= 1.0


def test_fp64_needs_the_dimension_factor():
    # in FP64 the same term without sqrt(m + n) falls below the loss: the
    # estimate keeps the factor there
    run = pr.gkl(_dense_problem(seed=1), 60, policy="none")
    m, n = 300, 200
    est = pr.OmegaEstimate(pr.EPS64, m + n, root=1.0)
    low = []
    for j in range(60):
        r = est.row_u(run["alpha"][j])
        est.push_u(run["alpha"][j], r, False)
        if j and 0 < run["loss_u"][j] < 1e-3:
            low.append(np.max(np.abs(r)) / run["loss_u"][j])
        r = est.row_v(run["beta"][j + 1])
        est.push_v(run["beta"][j + 1], r, False)
        if 0 < run["loss_v"][j] < 1e-3:
            low.append(np.max(np.abs(r)) / run["loss_v"][j])
    assert min(low) < 1.0
    assert _min_ratio(run)[0] >= 1.0


def test_ghosts_without_reorthogonalisation():
    A = _dense_problem(seed=3)
    k = 120
    top = np.linalg.svd(A, compute_uv=False)[0]
    counts = {}
    for policy in ("none", "partial", "full"):
        run = pr.gkl(A, k, policy=policy)
        s = pr.ritz(run["alpha"], run["beta"], k)[0]
        counts[policy] = int(np.sum(np.abs(s - top) <= 1e-8 * top))
    assert counts["none"] >= 2
    assert counts["partial"] == counts["full"] == 1


@pytest.mark.parametrize("case", ["dense", "config1", "config2", "later1", "later2"])
def test_partial_matches_full(case):
    if case == "dense":
        Y = _dense_problem(seed=4)
        sv = np.linalg.svd(Y, compute_uv=False)
        tau = 0.5 * (sv[5] + sv[6])
    else:
        Y, tau = _case(case)
    full = pr.decide(Y, tau, policy="full")
    part = pr.decide(Y, tau, policy="partial", eta=1e-10)
    assert full is not None and part is not None
    assert part["steps"] == full["steps"] and part["rank"] == full["rank"]
    np.testing.assert_allclose(part["sigma"], full["sigma"], rtol=1e-12)
    k = part["steps"]
    run = part["run"]
    assert max(run["loss_u"][:k].max(), run["loss_v"][:k].max()) < 1e-9
    assert part["reorth"] < 0.5 * part["vectors"]
    # the Ritz vectors of the values above tau: the same subspace
    for key in ("U", "V"):
        G = part[key].T @ full[key]
        np.testing.assert_allclose(np.abs(np.diag(G)), 1.0, atol=1e-9)


# ---------------------------------------------------------------- host code

@pytest.fixture(scope="module")
def capi(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    so = str(tmp_path_factory.mktemp("orth") / "liborth.so")
    subprocess.run([gxx, "-O2", "-std=c++17", "-shared", "-fPIC", f"-I{CSRC}",
                    os.path.join(ROOT, "tests", "orth_capi.cpp"), os.path.join(CSRC, "orth_estimate.cpp"),
                    "-o", so], check=True)
    lib = ctypes.CDLL(so)
    vp, d, i = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    for name, res, args in [("est_new", vp, [d, d]), ("est_push_u", d, [vp, d, i]), ("est_push_v", d, [vp, d, i]),
                            ("est_free", None, [vp]), ("sched_new", vp, [d, d, d, d, i]),
                            ("first_trigger", i, [dp, dp, i, d, d, d]),
                            ("exact_pattern", i, [dp, dp, i, d, d, d, ctypes.POINTER(ctypes.c_uint8)]),
                            ("sched_new_replay", vp, [d, d, d, d, i, ctypes.POINTER(ctypes.c_uint8), i, d]),
                            ("sched_decide", i, [vp, i]), ("sched_advance", i, [vp, dp, dp, i]),
                            ("sched_growth", d, [vp]), ("sched_growth_seen", d, [vp]), ("sched_free", None, [vp])]:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def test_host_estimate_equals_oracle(capi):
    Y, _ = _kick_iterate(1)
    m, n = Y.shape
    run = pr.gkl(Y, 60, policy="partial", eta=1e-10)
    e = capi.est_new(pr.EPS64, np.sqrt(m + n))
    try:
        for j in range(60):
            got_u = capi.est_push_u(e, run["alpha"][j], int(run["reorth_u"][j]))
            got_v = capi.est_push_v(e, run["beta"][j + 1], int(run["reorth_v"][j]))
            assert got_u == pytest.approx(run["est_u"][j], rel=1e-12, abs=1e-300)
            assert got_v == pytest.approx(run["est_v"][j], rel=1e-12, abs=1e-300)
    finally:
        capi.est_free(e)


@pytest.mark.parametrize("case,lag", [("dense", 8), ("config1", 8), ("config2", 8), ("later1", 8), ("later2", 8),
                                      ("later2", 3)])
def test_host_schedule_in_closed_loop(capi, case, lag):
    # the solver checks the coefficients of every snapshot before its rank
    # decision; here every `lag` steps (two steps behind, as the device runs
    # ahead of the check) and once more at the end
    if case == "dense":
        Y = _dense_problem(seed=5)
        sv = np.linalg.svd(Y, compute_uv=False)
        tau = 0.5 * (sv[5] + sv[6])
    else:
        Y, tau = _case(case)
    m, n = Y.shape
    full = pr.decide(Y, tau, policy="full")
    k = full["steps"]
    s = capi.sched_new(1e-10, pr.EPS64, np.sqrt(m + n), 8.0, 0)
    dp = ctypes.POINTER(ctypes.c_double)
    verdicts = []

    def check(alpha, beta, j):
        a = np.ascontiguousarray(alpha, dtype=np.float64)
        b = np.ascontiguousarray(beta, dtype=np.float64)
        verdicts.append(capi.sched_advance(s, a.ctypes.data_as(dp), b.ctypes.data_as(dp), j))

    try:
        def on_step(j, alpha, beta):
            if j % lag == 0 and j > 2:
                check(alpha, beta, j - 2)

        run = pr.gkl(Y, k, policy="given", decide=lambda h: capi.sched_decide(s, h), on_step=on_step)
        check(run["alpha"], run["beta"], k)
        growth = capi.sched_growth_seen(s)
    finally:
        capi.sched_free(s)
    loss = max(run["loss_u"].max(), run["loss_v"].max())
    orth = int(run["reorth_u"].sum() + run["reorth_v"].sum())
    assert orth < 0.6 * 2 * k
    # what the check must catch: a loss past semi-orthogonality is reported
    # (the solver then starts again with full reorthogonalisation)
    if loss >= np.sqrt(pr.EPS64):
        assert not all(verdicts)
    if case == "dense":
        return
    # on the completion iterates the prediction holds: no restart, the bases
    # stay semi-orthogonal and the triplets are the full method's
    assert all(verdicts) and loss < np.sqrt(pr.EPS64)
    sig, res, _, _ = pr.ritz(run["alpha"], run["beta"], k)
    r = full["rank"]
    np.testing.assert_allclose(sig[:r + 1], full["sigma"], rtol=1e-12)
    assert 1.0 < growth < 50.0


@pytest.mark.parametrize("case", ["config2", "later1", "later2"])
def test_host_schedule_fp32_in_closed_loop(capi, case):
    # the mixed form's setting: FP32 vectors, level 0.01 sqrt(u), c = 1
    Y, tau = _case(case)
    m, n = Y.shape
    full = pr.decide(Y, tau, policy="full")
    k = full["steps"]
    s = capi.sched_new(0.01 * np.sqrt(pr.EPS32), pr.EPS32, 1.0, 8.0, 0)
    dp = ctypes.POINTER(ctypes.c_double)
    verdicts = []

    def check(alpha, beta, j):
        a = np.ascontiguousarray(alpha, dtype=np.float64)
        b = np.ascontiguousarray(beta, dtype=np.float64)
        verdicts.append(capi.sched_advance(s, a.ctypes.data_as(dp), b.ctypes.data_as(dp), j))

    try:
        run = pr.gkl(Y, k, policy="given", store="f32", decide=lambda h: capi.sched_decide(s, h),
                     on_step=lambda j, a, b: check(a, b, j - 2) if j % 8 == 0 else None)
        check(run["alpha"], run["beta"], k)
    finally:
        capi.sched_free(s)
    assert all(verdicts)
    assert max(run["loss_u"].max(), run["loss_v"].max()) < np.sqrt(pr.EPS32)
    assert int(run["reorth_u"].sum() + run["reorth_v"].sum()) < 0.9 * 2 * k
    sig = pr.ritz(run["alpha"], run["beta"], k)[0]
    r = full["rank"]
    np.testing.assert_allclose(sig[:r + 1], full["sigma"], rtol=1e-5)


def test_host_schedule_reports_a_level_past_semi_orthogonality(capi):
    # a level above sqrt(u) lets the schedule leave vectors alone past
    # semi-orthogonality: its check must say so (the solver then starts
    # again with every vector orthogonalised)
    Y, tau = _case("later2")
    m, n = Y.shape
    s = capi.sched_new(100.0 * np.sqrt(pr.EPS64), pr.EPS64, np.sqrt(m + n), 8.0, 0)
    dp = ctypes.POINTER(ctypes.c_double)
    verdicts = []

    def check(alpha, beta, j):
        a = np.ascontiguousarray(alpha, dtype=np.float64)
        b = np.ascontiguousarray(beta, dtype=np.float64)
        verdicts.append(capi.sched_advance(s, a.ctypes.data_as(dp), b.ctypes.data_as(dp), j))

    try:
        run = pr.gkl(Y, 111, policy="given", decide=lambda h: capi.sched_decide(s, h),
                     on_step=lambda j, a, b: check(a, b, j - 2) if j % 8 == 0 else None)
        check(run["alpha"], run["beta"], 111)
    finally:
        capi.sched_free(s)
    assert not all(verdicts)
    assert max(run["loss_u"].max(), run["loss_v"].max()) > np.sqrt(pr.EPS64) * 1e-3


def test_host_estimate_at_a_breakdown(capi):
    # a zero or non-finite coefficient (the recurrence broke down) counts as
    # total loss of orthogonality, and later estimates stay finite
    Y, _ = _kick_iterate(1)
    m, n = Y.shape
    run = pr.gkl(Y, 12, policy="full")
    for bad in (0.0, float("nan"), float("inf")):
        e = capi.est_new(pr.EPS64, np.sqrt(m + n))
        try:
            for j in range(5):
                capi.est_push_u(e, run["alpha"][j], 1)
                capi.est_push_v(e, run["beta"][j + 1], 1)
            assert capi.est_push_u(e, bad, 0) == 1.0
            assert capi.est_push_v(e, bad, 0) == 1.0
            for j in range(6, 10):
                for got in (capi.est_push_u(e, run["alpha"][j], 0), capi.est_push_v(e, run["beta"][j + 1], 0)):
                    assert np.isfinite(got) and got >= 0.0
        finally:
            capi.est_free(e)


def _closed_loop(capi, Y, k, hold, lag=8, pattern=None):
    m, n = Y.shape
    if pattern is None:
        s = capi.sched_new(1e-10, pr.EPS64, np.sqrt(m + n), 8.0, hold)
    else:
        pat = np.ascontiguousarray(pattern, dtype=np.uint8)
        s = capi.sched_new_replay(1e-10, pr.EPS64, np.sqrt(m + n), 8.0, hold,
                                  pat.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), len(pat),
                                  float(np.sqrt(pr.EPS64)))
    dp = ctypes.POINTER(ctypes.c_double)
    verdicts = []

    def check(alpha, beta, j):
        a = np.ascontiguousarray(alpha, dtype=np.float64)
        b = np.ascontiguousarray(beta, dtype=np.float64)
        verdicts.append(capi.sched_advance(s, a.ctypes.data_as(dp), b.ctypes.data_as(dp), j))

    try:
        run = pr.gkl(Y, k, policy="given", decide=lambda h: capi.sched_decide(s, h),
                     on_step=lambda j, a, b: check(a, b, j - 2) if j % lag == 0 else None)
        check(run["alpha"], run["beta"], k)
    finally:
        capi.sched_free(s)
    return run, verdicts


@pytest.mark.parametrize("cfg,first,second", [(1, 5, 6), (2, 3, 4)])
def test_host_hold_from_the_previous_iterate(capi, cfg, first, second):
    # the first trigger of the exact policy, replayed on one SVT iterate's
    # coefficients, is where the library lets the next iterate's schedule
    # start orthogonalising (less 8 half-steps): the next run stays
    # semi-orthogonal with the full method's values and orthogonalises fewer
    # vectors than without the hold
    Y1, tau = _later_iterate(cfg, first)
    Y2, _ = _later_iterate(cfg, second)
    m, n = Y1.shape
    k1 = pr.decide(Y1, tau, policy="full")["steps"]
    run1, _ = _closed_loop(capi, Y1, k1, 0)
    dp = ctypes.POINTER(ctypes.c_double)
    a = np.ascontiguousarray(run1["alpha"], dtype=np.float64)
    b = np.ascontiguousarray(run1["beta"], dtype=np.float64)
    ft = capi.first_trigger(a.ctypes.data_as(dp), b.ctypes.data_as(dp), k1, 1e-10, pr.EPS64, np.sqrt(m + n))
    # the same point as the oracle's exact policy on the same iterate
    ex = pr.decide(Y1, tau, policy="partial", eta=1e-10)["run"]
    R = np.empty(2 * len(ex["reorth_u"]), bool)
    R[0::2], R[1::2] = ex["reorth_u"], ex["reorth_v"]
    assert abs(ft - int(np.nonzero(R)[0][0])) <= 2
    full = pr.decide(Y2, tau, policy="full")
    k2 = full["steps"]
    held, verdicts = _closed_loop(capi, Y2, k2, max(0, ft - 8))
    plain, _ = _closed_loop(capi, Y2, k2, 0)
    assert all(verdicts)
    assert max(held["loss_u"].max(), held["loss_v"].max()) < np.sqrt(pr.EPS64)
    n_held = int(held["reorth_u"].sum() + held["reorth_v"].sum())
    n_plain = int(plain["reorth_u"].sum() + plain["reorth_v"].sum())
    assert n_held < n_plain
    sig = pr.ritz(held["alpha"], held["beta"], k2)[0]
    r = full["rank"]
    np.testing.assert_allclose(sig[:r + 1], full["sigma"], rtol=1e-12)


def _pattern(run):
    R = np.empty(2 * len(run["reorth_u"]), bool)
    R[0::2], R[1::2] = run["reorth_u"], run["reorth_v"]
    return R


def _exact_pattern(capi, run, k, m, n):
    dp = ctypes.POINTER(ctypes.c_double)
    a = np.ascontiguousarray(run["alpha"][:k], dtype=np.float64)
    b = np.ascontiguousarray(run["beta"][:k + 1], dtype=np.float64)
    out = np.zeros(2 * k, np.uint8)
    got = capi.exact_pattern(a.ctypes.data_as(dp), b.ctypes.data_as(dp), k, 1e-10, pr.EPS64, np.sqrt(m + n),
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    assert got == 2 * k
    return out.astype(bool)


@pytest.mark.parametrize("cfg,it", [(1, 5), (2, 3)])
def test_host_exact_pattern_equals_oracle(capi, cfg, it):
    # the exact policy replayed on a run's coefficients names the vectors the
    # oracle's exact policy orthogonalised in that run (its estimates come
    # from the same coefficients and the same decisions)
    Y, tau = _later_iterate(cfg, it)
    m, n = Y.shape
    ex = pr.decide(Y, tau, policy="partial", eta=1e-10)
    k = ex["steps"]
    R = _pattern(ex["run"])[:2 * k]
    assert R.any()
    np.testing.assert_array_equal(_exact_pattern(capi, ex["run"], k, m, n), R)


@pytest.mark.parametrize("cfg,it", [(1, 5), (2, 3)])
def test_host_exact_pattern_fp32_equals_oracle(capi, cfg, it):
    # the same with FP32 vectors (the mixed form): FP32's unit roundoff, no
    # sqrt(m + n) factor, the automatic level 0.1 sqrt(u)
    Y, tau = _later_iterate(cfg, it)
    m, n = Y.shape
    eta = 0.1 * np.sqrt(pr.EPS32)
    k = pr.decide(Y, tau, policy="full")["steps"]
    run = pr.gkl(Y, k, policy="partial", eta=eta, store="f32")
    R = _pattern(run)[:2 * k]
    assert R.any()
    dp = ctypes.POINTER(ctypes.c_double)
    a = np.ascontiguousarray(run["alpha"][:k], dtype=np.float64)
    b = np.ascontiguousarray(run["beta"][:k + 1], dtype=np.float64)
    out = np.zeros(2 * k, np.uint8)
    assert capi.exact_pattern(a.ctypes.data_as(dp), b.ctypes.data_as(dp), k, eta, pr.EPS32, 1.0,
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))) == 2 * k
    np.testing.assert_array_equal(out.astype(bool), R)


@pytest.mark.parametrize("cfg,first,second", [(1, 5, 6), (2, 3, 4)])
def test_host_replay_from_the_previous_iterate(capi, cfg, first, second):
    # the next SVT iterate's schedule follows the exact policy's pattern on
    # the previous iterate's coefficients two half-steps ahead, its
    # predictions guarding only semi-orthogonality: every check passes, the
    # run stays semi-orthogonal with the full method's values, every vector
    # the pattern names (shifted) is orthogonalised, and fewer vectors are
    # orthogonalised than with the hold alone
    Y1, tau = _later_iterate(cfg, first)
    Y2, _ = _later_iterate(cfg, second)
    m, n = Y1.shape
    k1 = pr.decide(Y1, tau, policy="full")["steps"]
    run1, _ = _closed_loop(capi, Y1, k1, 0)
    pat = _exact_pattern(capi, run1, k1, m, n)
    dp = ctypes.POINTER(ctypes.c_double)
    a = np.ascontiguousarray(run1["alpha"], dtype=np.float64)
    b = np.ascontiguousarray(run1["beta"], dtype=np.float64)
    hold = max(0, capi.first_trigger(a.ctypes.data_as(dp), b.ctypes.data_as(dp), k1, 1e-10, pr.EPS64,
                                     np.sqrt(m + n)) - 8)
    full = pr.decide(Y2, tau, policy="full")
    k2 = full["steps"]
    replayed, verdicts = _closed_loop(capi, Y2, k2, hold, pattern=pat)
    held, _ = _closed_loop(capi, Y2, k2, hold)
    assert all(verdicts)
    assert max(replayed["loss_u"].max(), replayed["loss_v"].max()) < np.sqrt(pr.EPS64)
    R = _pattern(replayed)
    lead = 2
    for h in np.nonzero(pat)[0]:
        if h - lead >= 1 and h - lead < len(R):
            assert R[h - lead]
    assert R.sum() < _pattern(held).sum()
    sig = pr.ritz(replayed["alpha"], replayed["beta"], k2)[0]
    r = full["rank"]
    np.testing.assert_allclose(sig[:r + 1], full["sigma"], rtol=1e-12)
