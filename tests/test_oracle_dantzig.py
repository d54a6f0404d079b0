"""The oracle's Dantzig-selector iteration (Section 3.3, eq. (3.10)) pinned to
what the mathematics fixes, without another implementation of it:

* E at least every |B_ij|: X = 0 is feasible, and the iteration returns it;
* the kick: the run from Y+- = 0 equals the kicked run shifted by k0;
* Theorem 4.4 (0 < delta < 2 / L^2, L^2 = 2 for the two stacked constraint
  maps): the limit satisfies the KKT conditions of problem (3.8) with
  A = P_Omega -- feasibility, nonnegative multipliers, complementary
  slackness, X = D_tau(Y+ - Y-) checked with LAPACK's SVD -- which, the
  objective being strongly convex, make it the unique solution; random
  feasible perturbations do not lower the objective;
* E = 0: the constraint is P_Omega X = P_Omega B, so the limit equals the
  equality iteration's (Algorithm 1 run to convergence with the same tau);
* the Figure 3 workload's noise ratio is the closed form
  0.1 E|M_ij| / rms(M_ij) ~ 0.1 sqrt(2 / pi) (the paper prints 0.780 for
  about 0.078).
"""
import numpy as np
import pytest

import oracle
import workload
from oracle.dantzig import soft_threshold, svt_dantzig
from tests.helpers import rel_diff_factored


def _small(seed=0, m=30, n=24, r=2, frac=0.6, noise=0.1):
    p = workload.gaussian_lowrank(m, n, r, int(frac * m * n), seed, noise_sigma=noise)
    return p


def _dense(p, y):
    Y = np.zeros((p.m, p.n))
    Y[p.rows, p.cols] = y
    return Y


def test_large_tolerance_gives_zero():
    p = _small()
    E = float(np.max(np.abs(p.vals)))
    for kick in (True, False):
        d = svt_dantzig(p.m, p.n, p.rows, p.cols, p.vals, E, p.tau, p.delta, p.eps, 50, p.incr, kick=kick)
        assert d["iters"] == 1 and d["status"] == "ok" and d["k0"] == 0
        assert d["ranks"] == [0] and d["U"].shape[1] == 0 and d["residuals"] == [0.0]


def test_kick_equals_unskipped_run_shifted():
    p = _small(seed=3)
    E = 0.05
    a = svt_dantzig(p.m, p.n, p.rows, p.cols, p.vals, E, p.tau, p.delta, p.eps, 400, p.incr, kick=True)
    b = svt_dantzig(p.m, p.n, p.rows, p.cols, p.vals, E, p.tau, p.delta, p.eps, 400 + a["k0"], p.incr,
                    kick=False)
    k0 = a["k0"]
    assert k0 >= 1
    assert b["ranks"][:k0] == [0] * k0 and b["ranks"][k0] > 0
    assert b["ranks"][k0:] == a["ranks"] and b["iters"] == a["iters"] + k0
    np.testing.assert_allclose(b["residuals"][k0:], a["residuals"], rtol=1e-9)
    assert rel_diff_factored(b["U"], b["V"], a["U"], a["V"]) <= 1e-9


def _kkt_run(p, E, delta, maxiter=20000):
    return svt_dantzig(p.m, p.n, p.rows, p.cols, p.vals, E, p.tau, delta, 1e-13, maxiter, p.incr,
                       keep_multipliers=True)


@pytest.mark.parametrize("seed,E", [(1, 0.1), (2, 0.3)])
def test_kkt_conditions_at_the_limit(seed, E):
    p = _small(seed=seed)
    p.tau = 20.0
    d = _kkt_run(p, E, 0.9)
    X = d["U"] @ d["V"].T
    x = X[p.rows, p.cols]
    b = p.vals
    yp, ym = d["yp"], d["ym"]
    scale = np.max(np.abs(b))
    # feasibility
    assert np.all(np.abs(x - b) <= E + 1e-9 * scale)
    # nonnegative multipliers, complementary slackness
    assert np.all(yp >= 0) and np.all(ym >= 0)
    act_p = yp > 1e-9 * np.max(yp + ym)
    act_m = ym > 1e-9 * np.max(yp + ym)
    assert np.all(np.abs((b - x)[act_p] - E) <= 1e-8 * scale)
    assert np.all(np.abs((x - b)[act_m] - E) <= 1e-8 * scale)
    assert act_p.any() and act_m.any()
    # stationarity: X = D_tau(Y+ - Y-), the shrinkage taken with LAPACK
    Uf, s, Vt = np.linalg.svd(_dense(p, yp - ym), full_matrices=False)
    w = np.maximum(s - p.tau, 0.0)
    Xref = (Uf * w) @ Vt
    assert np.linalg.norm(X - Xref) <= 1e-8 * np.linalg.norm(Xref)
    # the objective does not drop under feasible perturbations
    f = lambda Z: p.tau * np.linalg.svd(Z, compute_uv=False).sum() + 0.5 * np.sum(Z * Z)  # noqa: E731
    rng = np.random.default_rng(seed)
    f0 = f(X)
    for _ in range(50):
        Z = X + 1e-3 * rng.standard_normal(X.shape)
        z = Z[p.rows, p.cols]
        z = np.clip(z, b - E, b + E)   # back into the feasible box on Omega
        Z[p.rows, p.cols] = z
        assert f(Z) >= f0 - 1e-9 * abs(f0)


def test_zero_tolerance_has_the_equality_limit():
    p = _small(seed=4)
    p.tau = 20.0
    d = _kkt_run(p, 0.0, 0.9)
    e = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, 0.9, 1e-13, 20000, p.incr)
    assert d["status"] == "ok" and e["status"] == "ok"
    assert rel_diff_factored(d["U"], d["V"], e["U"], e["V"]) <= 1e-8


def test_sparse_partial_svd_route_matches_dense():
    p = workload.gaussian_lowrank(120, 100, 3, 5000, 6, noise_sigma=0.05)
    E = 0.05
    a = svt_dantzig(p.m, p.n, p.rows, p.cols, p.vals, E, p.tau, p.delta * 0.5, p.eps, 300, p.incr)
    c = svt_dantzig(p.m, p.n, p.rows, p.cols, p.vals, E, p.tau, p.delta * 0.5, p.eps, 300, p.incr,
                    partial="sparse")
    assert a["iters"] == c["iters"] and a["ranks"] == c["ranks"] and a["s_hist"] == c["s_hist"]
    np.testing.assert_allclose(c["residuals"], a["residuals"], rtol=1e-9)
    assert rel_diff_factored(c["U"], c["V"], a["U"], a["V"]) <= 1e-9


def test_soft_threshold():
    np.testing.assert_array_equal(soft_threshold([3.0, -3.0, 0.5, -0.5, 1.0], 1.0), [2.0, -2.0, 0.0, 0.0, 0.0])


def test_figure3_noise_ratio():
    p = workload.dantzig_fig3(seed=0)
    ratio = np.linalg.norm(p.vals - p.clean) / np.linalg.norm(p.clean)
    closed = 0.1 * np.mean(np.abs(p.clean)) / np.sqrt(np.mean(p.clean ** 2))
    assert abs(ratio - closed) <= 0.01 * closed
    assert abs(closed - 0.1 * np.sqrt(2 / np.pi)) <= 0.005
