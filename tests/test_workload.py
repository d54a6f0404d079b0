"""The seeded generators: Omega is a set, uniform, reproducible, and the sizes
follow the paper's arithmetic (d_r = r(2n - r), Section 1.1; Table 1)."""
import os

import numpy as np
import pytest

import workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_shapes.txt")


def _table1():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        n, r, c, frac, iters, err = line.split()
        rows.append((int(n), int(r), int(c), float(frac), int(iters), float(err)))
    return rows


def test_table1_sampling_fraction_arithmetic():
    # m = (m/d_r) * r (2n - r); the printed m/n^2 is that ratio rounded
    rows = _table1()
    assert len(rows) == 12
    for n, r, c, frac, _, _ in rows:
        m = c * workload.degrees_of_freedom(n, n, r)
        printed_digits = len(str(frac).split(".")[1])
        assert round(m / n ** 2, printed_digits) == pytest.approx(frac, abs=10 ** -printed_digits)


def test_table1_headline_claims():
    rows = _table1()
    assert all(it < 200 for *_, it, _ in rows)          # "fewer than 200 SVT iterations"
    assert all(err < 2e-4 for *_, err in rows)          # "all less than 2e-4"


def test_omega_is_a_uniform_set_and_reproducible():
    p = workload.gaussian_lowrank(300, 200, 4, 9000, seed=3)
    lin = p.rows.astype(np.int64) * p.n + p.cols
    assert np.unique(lin).shape[0] == p.nnz
    assert np.all(np.diff(lin) > 0)                      # row-major sorted
    assert p.rows.min() >= 0 and p.rows.max() < p.m and p.cols.max() < p.n
    q = workload.gaussian_lowrank(300, 200, 4, 9000, seed=3)
    assert np.array_equal(p.rows, q.rows) and np.array_equal(p.vals, q.vals)
    # rows get about nnz/m samples each (binomial, no skew)
    counts = np.bincount(p.rows, minlength=p.m)
    assert abs(counts.mean() - 30.0) < 1e-9 and counts.std() < 10
    np.testing.assert_allclose(p.vals, (p.ML @ p.MR.T)[p.rows, p.cols], rtol=1e-12, atol=1e-12)


def test_configs_parameters():
    p = workload.config(1)
    assert (p.m, p.n, p.r, p.nnz) == (400, 400, 10, 47400)
    assert p.tau == 2000.0 and abs(p.delta - 1.2 * 400 * 400 / 47400) < 1e-12
    assert p.eps == 1e-4 and p.maxiter == 500 and p.incr == 5


def test_serving_trace_respects_fill_cap():
    trace = workload.serving_trace(200, seed=1, rate=5.0)
    times = [t for t, _ in trace]
    assert all(b >= a for a, b in zip(times, times[1:]))
    for _, s in trace:
        assert 500 <= s["m"] <= 8000 and 500 <= s["n"] <= 8000
        assert s["r"] in (5, 10, 20, 50)
        assert s["nnz"] <= 0.6 * s["m"] * s["n"]
        assert 3 * s["r"] * (s["m"] + s["n"] - s["r"]) <= s["nnz"] + 1
        assert s["nnz"] <= 6 * s["r"] * (s["m"] + s["n"] - s["r"])


def test_serving_trace_table1_pairs():
    trace = workload.serving_trace(100, seed=2, mn_range=(1000, 8000),
                                   pairs=workload.TABLE1_RANK_OVERSAMPLING, max_aspect=1.5)
    for _, s in trace:
        c = {10: 6, 50: 5, 100: 4}[s["r"]]
        assert s["nnz"] == int(c * s["r"] * (s["m"] + s["n"] - s["r"]))
        assert max(s["m"], s["n"]) <= 1.5 * min(s["m"], s["n"])


def test_stored_oracle_result_matches_current_generator():
    # the stored 400 x 400 oracle run must belong to today's generator: its
    # first two iterations are recomputed here
    import oracle
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "oracle_config1.npz"))
    p = workload.config(1)
    out = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, 2, p.incr)
    assert out["k0"] == int(g["k0"])
    assert list(out["ranks"]) == list(g["ranks"][:2])
    np.testing.assert_allclose(out["residuals"], g["residuals"][:2], rtol=1e-12)
