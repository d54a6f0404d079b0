"""HIP path against the CPU oracle (needs an MI355X).

Each test calls the C ABI through the binding and compares with the oracle on
the same seeded inputs.  Tolerances for the plain FP64 path:
  * sparse products and the sampled update: entrywise relative 1e-12 (sums of
    at most a few hundred products, each exact to 2^-53);
  * Ritz values: 1e-11 relative to sigma_1 (Lanczos residual bound 1e-12);
  * whole solves: identical rank sequence and iteration count, residual history
    within 1e-8 relative, final ||X - X_oracle||_F / ||X_oracle||_F <= 1e-8.
"""
import os

import numpy as np
import pytest

import oracle
import workload
from paper_0810_3286_amd import svt as B
from tests.helpers import gpu_case, rel_diff_factored

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _create(p, **kw):
    prm = B.svt_params_default(p.m, p.n, p.nnz)
    prm.tau, prm.delta, prm.eps = p.tau, p.delta, p.eps
    prm.maxiter, prm.incr = p.maxiter, p.incr
    for k, v in kw.items():
        setattr(prm, k, v)
    return B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)


SMALL = [
    # (m, n, r, nnz, seed): square, tall, wide, ragged sizes, a near-dense case
    (120, 120, 3, 4000, 0),
    (157, 93, 4, 5200, 1),
    (61, 203, 2, 3100, 2),
    (33, 29, 2, 700, 3),
]


@pytest.mark.parametrize("mode", [1, 2])   # 1: x gathered from memory, 2: staged in LDS
@pytest.mark.parametrize("case", SMALL + [(400, 400, 10, 47400, 0), (1000, 777, 5, 60000, 4)])
def test_sparse_products(case, mode):
    m, n, r, nnz, seed = case
    gpu_case(f"spmv {case} mode {mode}")
    p = workload.gaussian_lowrank(m, n, r, nnz, seed, shuffle=True)
    y = workload.dense_random_iterate(p, seed + 10)
    rng = np.random.default_rng(seed + 20)
    x = rng.standard_normal(n)
    u = rng.standard_normal(m)
    h = _create(p, spmv_mode=mode)
    try:
        B.svt_set_iterate(h, y)
        got = B.svt_apply(h, x, m, trans=0)
        gotT = B.svt_apply(h, u, n, trans=1)
        plan = (B.svt_spmv_plan(h, 0), B.svt_spmv_plan(h, 1))
    finally:
        B.svt_destroy(h)
    # FP64 x of these sizes fits LDS whole: mode 2 stages it in one segment
    assert plan == ((0, 0) if mode == 1 else (1, 1))
    ref = oracle.apply_sparse(m, n, p.rows, p.cols, y, x)
    refT = oracle.apply_sparse(m, n, p.rows, p.cols, y, u, trans=True)
    scale = oracle.apply_sparse(m, n, p.rows, p.cols, np.abs(y), np.abs(x))
    scaleT = oracle.apply_sparse(m, n, p.rows, p.cols, np.abs(y), np.abs(u), trans=True)
    assert np.all(np.abs(got - ref) <= 1e-14 * 64 * scale + 1e-300)
    assert np.all(np.abs(gotT - refT) <= 1e-14 * 64 * scaleT + 1e-300)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_sparse_products_full_size_30000(precision, mode):
    # staged in LDS (mode 2), FP64 x takes two column segments at n = 30000,
    # FP32 x (mixed form) one; mode 1 gathers x from memory
    gpu_case(f"spmv 30000^2 precision {precision} mode {mode}")
    p = workload.config(4)
    y = workload.dense_random_iterate(p, 5)
    rng = np.random.default_rng(6)
    x = rng.standard_normal(p.n)
    h = _create(p, precision=precision, spmv_mode=mode)
    try:
        B.svt_set_iterate(h, y)
        got = B.svt_apply(h, x, p.m, trans=0)
        gotT = B.svt_apply(h, x, p.n, trans=1)
        plan = (B.svt_spmv_plan(h, 0), B.svt_spmv_plan(h, 1))
    finally:
        B.svt_destroy(h)
    # the kernel asked for is the one that ran (no silent fall-back)
    want = 0 if mode == 1 else (2 if precision == 0 else 1)
    assert plan == (want, want)
    # rows sampled one by one by the oracle's plain definition
    rows = rng.choice(p.m, 300, replace=False)
    sel = np.isin(p.rows, rows)
    if precision == 1:  # inputs rounded to FP32, FP32 accumulation
        y = y.astype(np.float32).astype(np.float64)
        x = x.astype(np.float32).astype(np.float64)
    tol = 1e-12 if precision == 0 else 2e-5
    ref = oracle.apply_sparse(p.m, p.n, p.rows[sel], p.cols[sel], y[sel], x)
    scale = oracle.apply_sparse(p.m, p.n, p.rows[sel], p.cols[sel], np.abs(y[sel]), np.abs(x))
    assert np.all(np.abs(got[rows] - ref[rows]) <= tol * scale[rows])
    cols = rng.choice(p.n, 300, replace=False)
    selc = np.isin(p.cols, cols)
    refT = oracle.apply_sparse(p.m, p.n, p.rows[selc], p.cols[selc], y[selc], x, trans=True)
    scaleT = oracle.apply_sparse(p.m, p.n, p.rows[selc], p.cols[selc], np.abs(y[selc]), np.abs(x), trans=True)
    assert np.all(np.abs(gotT[cols] - refT[cols]) <= tol * scaleT[cols])


@pytest.mark.parametrize("case", SMALL + [(400, 400, 10, 47400, 0)])
@pytest.mark.parametrize("rank", [0, 1, 7, 10, 12, 16, 20, 40, 70, 100])
def test_sample_update(case, rank):
    m, n, r, nnz, seed = case
    gpu_case(f"sample_update {case} rank {rank}")
    p = workload.gaussian_lowrank(m, n, r, nnz, seed, shuffle=True)
    y = workload.dense_random_iterate(p, seed + 11)
    rng = np.random.default_rng(seed + 30)
    U = rng.standard_normal((m, rank))
    V = rng.standard_normal((n, rank))
    delta = 1.7
    h = _create(p)
    try:
        B.svt_set_iterate(h, y)
        res2 = B.svt_sample_update(h, U, V, delta)
        y_csr = B.svt_get_iterate(h, p.nnz, 0)
        y_csc = B.svt_get_iterate(h, p.nnz, 1)
    finally:
        B.svt_destroy(h)
    x = oracle.sampled_entries(U, V, p.rows, p.cols)
    e = p.vals - x
    np.testing.assert_allclose(res2, np.sum(e * e), rtol=1e-12)
    np.testing.assert_allclose(y_csr, y + delta * e, rtol=1e-12, atol=1e-12 * np.abs(y).max())
    assert np.array_equal(y_csr, y_csc)  # both compressed copies identical bit for bit


@pytest.mark.parametrize("case", SMALL + [(400, 400, 10, 47400, 0)])
@pytest.mark.parametrize("rank", [1, 10, 12, 16, 20, 40, 70, 100])
def test_sample_update_mixed(case, rank):
    # the mixed form's pass (FP32 factors, values and products; compensated
    # FP32 sum of e^2 promoted to FP64): every kernel variant (factor rows in
    # 8, 16, 32 or 64 registers, or read from memory) against the oracle's
    # plain definition on the FP32-rounded inputs
    m, n, r, nnz, seed = case
    gpu_case(f"sample_update mixed {case} rank {rank}")
    p = workload.gaussian_lowrank(m, n, r, nnz, seed, shuffle=True)
    y = workload.dense_random_iterate(p, seed + 11)
    rng = np.random.default_rng(seed + 31)
    U = rng.standard_normal((m, rank))
    V = rng.standard_normal((n, rank))
    delta = 1.7
    h = _create(p, precision=B.SVT_MIXED)
    try:
        B.svt_set_iterate(h, y)
        res2 = B.svt_sample_update(h, U, V, delta)
        y_csr = B.svt_get_iterate(h, p.nnz, 0)
        y_csc = B.svt_get_iterate(h, p.nnz, 1)
    finally:
        B.svt_destroy(h)
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)  # noqa: E731
    Uf, Vf, Mf, yf = f32(U), f32(V), f32(p.vals), f32(y)
    x = oracle.sampled_entries(Uf, Vf, p.rows, p.cols)
    e = Mf - x
    # FP32 rounding of the rank-r dot products: ~r 2^-24 sum |u_l v_l|
    mag = oracle.sampled_entries(np.abs(Uf), np.abs(Vf), p.rows, p.cols) + np.abs(Mf)
    err = (rank + 2) * 2.0 ** -23 * mag
    assert np.all(np.abs((y_csr - yf) / delta - e) <= err / 1.0 + 4 * 2.0 ** -24 * np.abs(yf + delta * e) / delta)
    assert abs(res2 - np.sum(e * e)) <= 2 * np.sum(np.abs(e) * err) + 1e-6 * np.sum(e * e)
    assert np.array_equal(y_csr, y_csc)


@pytest.mark.parametrize("case", SMALL)
def test_partial_svd_against_jacobi(case):
    m, n, r, nnz, seed = case
    gpu_case(f"partial_svd {case}")
    p = workload.gaussian_lowrank(m, n, r, nnz, seed)
    y = workload.dense_random_iterate(p, seed + 12)
    count = min(8, min(m, n))
    h = _create(p)
    try:
        B.svt_set_iterate(h, y)
        sig, U, V, steps = B.svt_partial_svd(h, count, m, n)
    finally:
        B.svt_destroy(h)
    Yd = np.zeros((m, n))
    Yd[p.rows, p.cols] = y
    Uo, so, Vo = oracle.top_triplets_dense(Yd, count)
    np.testing.assert_allclose(sig, so, rtol=0, atol=1e-11 * so[0])
    # vectors up to sign, for well separated values
    for i in range(count):
        gap = min([abs(so[i] - so[j]) for j in range(count) if j != i] + [so[0]])
        if gap > 1e-3 * so[0]:
            assert abs(abs(U[:, i] @ Uo[:, i]) - 1) <= 1e-9
            assert abs(abs(V[:, i] @ Vo[:, i]) - 1) <= 1e-9
    assert np.linalg.norm(Yd @ V - U * sig) <= 1e-10 * so[0]


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
@pytest.mark.parametrize("count", [17, 40, 64, 70, 130])
def test_partial_svd_wide_factors(count, precision):
    # Ritz vectors of 17 to 130 columns: one to four 16-column tiles per
    # workgroup and more than one group of 64 output columns (the matrix-core
    # product of the basis with the small SVD's vectors); 333 rows: a ragged
    # last group of 64 rows
    gpu_case(f"partial_svd {count} triplets precision {precision}")
    m, n = 333, 290
    p = workload.gaussian_lowrank(m, n, 5, 40000, 9)
    y = workload.dense_random_iterate(p, 21)
    prm = B.svt_params_default(p.m, p.n, p.nnz)
    prm.precision = precision
    h = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
    try:
        B.svt_set_iterate(h, y)
        sig, U, V, steps = B.svt_partial_svd(h, count, m, n)
    finally:
        B.svt_destroy(h)
    Yd = np.zeros((m, n))
    Yd[p.rows, p.cols] = y
    Uo, so, Vo = oracle.top_triplets_dense(Yd, count)
    tol = 1e-11 if precision == B.SVT_FP64 else 2e-6
    np.testing.assert_allclose(sig, so, rtol=0, atol=tol * so[0])
    # Y v_i = sigma_i u_i and orthonormal factors, column by column
    assert np.linalg.norm(Yd @ V - U * sig) <= 10 * tol * so[0] * np.sqrt(count)
    np.testing.assert_allclose(U.T @ U, np.eye(count), atol=100 * tol)
    np.testing.assert_allclose(V.T @ V, np.eye(count), atol=100 * tol)


@pytest.mark.parametrize("case", SMALL + [(400, 400, 10, 47400, 0)])
def test_kick(case):
    m, n, r, nnz, seed = case
    gpu_case(f"kick {case}")
    p = workload.gaussian_lowrank(m, n, r, nnz, seed)
    h = _create(p)
    try:
        s1, k0 = B.svt_kick(h)
        y = B.svt_get_iterate(h, p.nnz, 0)
    finally:
        B.svt_destroy(h)
    Pm = np.zeros((m, n))
    Pm[p.rows, p.cols] = p.vals
    so = oracle.jacobi_svd(Pm)[1][0]
    assert abs(s1 - so) <= 1e-11 * so
    assert k0 == oracle.k0_kick(p.tau, p.delta, so)
    np.testing.assert_allclose(y, k0 * p.delta * p.vals, rtol=1e-15)


def _compare_solves(g, o, iters_exact=True):
    assert g["status"] == (B.SVT_OK if o["status"] == "ok" else B.SVT_NOT_CONVERGED)
    assert g["info"]["k0"] == o["k0"]
    if iters_exact:
        assert g["info"]["iters"] == o["iters"]
        assert list(g["ranks"]) == list(o["ranks"])
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=1e-8)
    d = rel_diff_factored(g["U"], g["V"], o["U"], o["V"])
    assert d <= 1e-8, d


# solves that converge: the iteration is then contractive near its limit, so
# the two implementations' trajectories stay within rounding of each other
SOLVE_CASES = [
    (150, 150, 4, 7000, 6),
    (90, 260, 3, 8000, 3),     # wide: bidiagonalisation runs on Y^T
    (260, 90, 3, 8000, 5),
    (33, 29, 2, 700, 3),       # 73% observed
]


@pytest.mark.parametrize("case", SOLVE_CASES)
def test_solve_parity_small(case):
    m, n, r, nnz, seed = case
    gpu_case(f"solve {case}")
    p = workload.gaussian_lowrank(m, n, r, nnz, seed, maxiter=300, shuffle=True)
    from paper_0810_3286_amd import solve
    g = solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta, eps=p.eps,
              maxiter=p.maxiter, incr=p.incr)
    o = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps,
                         p.maxiter, p.incr)
    _compare_solves(g, o)
    assert list(g["s_hist"]) == list(o["s_hist"])


@pytest.mark.parametrize("m,n,sig", [
    (30, 20, [400.0, 150.0, 60.0, 20.0]),
    (16, 24, [300.0, 90.0, 45.0]),
    (12, 12, [500.0, 480.0, 30.0, 29.0, 5.3]),
    (30, 20, [90.0, 50.0, 21.0]),
])
def test_full_observation_closed_form(m, n, sig):
    # Omega = every entry: the run has a closed form (see test_oracle_svt)
    from tests.test_oracle_svt import full_observation_closed_form
    from paper_0810_3286_amd import solve
    gpu_case(f"fullobs {m}x{n}")
    sig = np.array(sig)
    p, U, _, V = workload.full_observation(m, n, sig, seed=m + n)
    g = solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta, eps=p.eps,
              maxiter=p.maxiter, incr=p.incr)
    ref = full_observation_closed_form(sig, p.tau, p.delta, p.eps, p.maxiter)
    assert g["info"]["k0"] == ref["k0"]
    assert g["info"]["iters"] == ref["iters"]
    assert list(g["ranks"]) == ref["ranks"]
    np.testing.assert_allclose(g["residuals"], ref["residuals"], rtol=1e-8, atol=1e-12)
    d = rel_diff_factored(g["U"], g["V"], U * ref["x"], V)
    assert d <= 1e-10


def test_solve_parity_400():
    # 400 x 400, rank 10, |Omega| = 6 d_r, FP64: the oracle's run is stored
    gpu_case("solve 400^2 vs stored oracle")
    p = workload.config(1)
    gold = np.load(os.path.join(GOLDEN, "oracle_config1.npz"))
    from paper_0810_3286_amd import solve
    g = solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta, eps=p.eps,
              maxiter=p.maxiter, incr=p.incr)
    o = dict(status="ok", k0=int(gold["k0"]), iters=int(gold["iters"]), ranks=list(gold["ranks"]),
             residuals=gold["residuals"], U=gold["U"], V=gold["V"])
    _compare_solves(g, o)
    assert list(g["s_hist"]) == list(gold["s_hist"])
    X_rel = rel_diff_factored(g["U"], g["V"], p.ML, p.MR)
    assert X_rel < 2e-4  # Table 1: relative errors below 2e-4


def test_solve_repeatable_and_history():
    gpu_case("solve repeat")
    p = workload.gaussian_lowrank(150, 150, 4, 7000, 6)  # converges (130 iterations)
    h = _create(p)
    try:
        st1, i1 = B.svt_solve(h)
        U1, w1, V1 = B.svt_factors(h, p.m, p.n)
        st2, i2 = B.svt_solve(h)
        U2, w2, V2 = B.svt_factors(h, p.m, p.n)
        hist = B.svt_history(h)
        pred = B.svt_predict(h, p.rows[:50], p.cols[:50])
    finally:
        B.svt_destroy(h)
    assert st1 == st2 == B.SVT_OK and i1.iters == i2.iters
    assert np.array_equal(U1, U2) and np.array_equal(V1, V2)   # deterministic
    assert len(hist["ranks"]) == i1.iters
    assert np.all(np.diff(hist["ranks"]) >= 0)
    np.testing.assert_allclose(pred, np.sum(U1[p.rows[:50]] * V1[p.cols[:50]], axis=1), rtol=1e-12)


def test_maxiter_reports_not_converged():
    gpu_case("maxiter=3")
    p = workload.gaussian_lowrank(100, 90, 3, 3000, 8, maxiter=3)
    from paper_0810_3286_amd import solve
    g = solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta, eps=p.eps, maxiter=3)
    assert g["status"] == B.SVT_NOT_CONVERGED and g["info"]["iters"] == 3


def test_unkicked_solve_matches_oracle():
    gpu_case("solve kick=0")
    p = workload.gaussian_lowrank(80, 70, 2, 2500, 9, maxiter=300)
    from paper_0810_3286_amd import solve
    g = solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta, eps=p.eps,
              maxiter=p.maxiter, kick=0)
    o = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps,
                         p.maxiter, p.incr, kick=False)
    _compare_solves(g, o)


@pytest.mark.parametrize("precision", [0, 1])
def test_partial_svd_across_basis_growth(precision):
    # 70 triplets need more than 64 bidiagonalisation steps: the bases grow
    # mid-run and the pending vector's norm partials must survive the move
    gpu_case(f"partial_svd growth precision {precision}")
    p = workload.gaussian_lowrank(300, 250, 5, 30000, 21)
    y = workload.dense_random_iterate(p, 22)
    h = _create(p, precision=precision)
    try:
        B.svt_set_iterate(h, y)
        sig, U, V, steps = B.svt_partial_svd(h, 70, p.m, p.n)
    finally:
        B.svt_destroy(h)
    assert steps > 64
    Yd = np.zeros((p.m, p.n))
    Yd[p.rows, p.cols] = y
    so = oracle.top_triplets_dense(Yd, 70)[1]
    tol = 1e-11 if precision == 0 else 2e-5
    np.testing.assert_allclose(sig, so, rtol=0, atol=tol * so[0])


@pytest.mark.parametrize("m", [16384, 16640])
@pytest.mark.parametrize("precision", [0, 1])
def test_partial_svd_row_block_boundary(m, precision):
    # 256 row blocks of 64 rows (m = 16384) take the 64-row-slot passes of
    # the sparse product once the basis reaches 64 columns; 65 rows (m =
    # 16640) take the 128-row-slot passes.  Both against the oracle.
    gpu_case(f"partial_svd {m} x 200, 70 triplets, precision {precision}")
    p = workload.gaussian_lowrank(m, 200, 5, 200000, 31)
    y = workload.dense_random_iterate(p, 32)
    h = _create(p, precision=precision)
    try:
        B.svt_set_iterate(h, y)
        sig, U, V, steps = B.svt_partial_svd(h, 70, p.m, p.n)
    finally:
        B.svt_destroy(h)
    assert steps > 64
    Yd = np.zeros((p.m, p.n))
    Yd[p.rows, p.cols] = y
    so = oracle.top_triplets_dense(Yd, 70)[1]
    tol = 1e-11 if precision == 0 else 2e-5
    np.testing.assert_allclose(sig, so, rtol=0, atol=tol * so[0])


def test_mixed_hard_request_stays_finite():
    # a request whose singular values cluster at tau needs long
    # bidiagonalisations every iteration (it does not converge in 60)
    gpu_case("mixed 700x500 hard request")
    p = workload.gaussian_lowrank(700, 500, 5, 30000, 11, shuffle=True)
    from paper_0810_3286_amd import solve
    g = solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta, eps=p.eps,
              maxiter=60, incr=p.incr, precision=B.SVT_MIXED)
    assert g["status"] == B.SVT_NOT_CONVERGED
    assert np.all(np.isfinite(g["residuals"])) and max(g["gkl_steps"]) > 64


def test_step_cap_error_reports_progress():
    # the hard request needs more than 64 bidiagonalisation steps after a
    # few iterations: with the cap at 64 the solve fails with SVT_ELANCZOS,
    # and the info still reports the iterations completed before it
    gpu_case("step cap 64 on the 700x500 hard request")
    p = workload.gaussian_lowrank(700, 500, 5, 30000, 11, shuffle=True)
    h = _create(p, maxiter=60, precision=B.SVT_MIXED, lanczos_maxsteps=64)
    try:
        with pytest.raises(B.SvtError) as ei:
            B.svt_solve(h)
        hist = B.svt_history(h)
    finally:
        B.svt_destroy(h)
    e = ei.value
    assert e.status == B.SVT_ELANCZOS and e.info is not None
    assert e.info.status == B.SVT_ELANCZOS
    assert e.info.iters == len(hist["ranks"]) >= 1
    assert np.all(np.isfinite(hist["residuals"])) and max(hist["gkl_steps"]) <= 64
