"""The oracle's own sensitivity to rounding on the 5000 x 5000, rank-10,
|Omega| = 5 d_r workload, from the stored runs of
``tests/golden/make_rounding_spread.py`` (tier C, 21 runs whose inputs or
start vectors differ only by rounding: one unit in the last place of every
observed value, or other seeds of the partial SVD's start vectors).

It shows, with the oracle alone, what the GPU comparison of complete runs at
this size must allow for: the histories agree to rounding for 50
iterations, the difference then grows by orders of magnitude (the iterate's
11th and 12th singular values hover around tau late in the run), and the
runs stop at different iterations with final X a few 1e-5 apart.
"""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _spread():
    return np.load(os.path.join(GOLDEN, "oracle_config2_spread.npz"))


def test_rounding_regime_then_amplification():
    g = _spread()
    R = g["residuals"]
    base = R[0]
    rel = np.abs(R[1:] - base) / base
    assert np.nanmax(rel[:, :50]) <= 1e-12          # rounding-level agreement
    assert np.nanmax(rel[:, 140:150]) >= 1e-3       # amplified to the residual's own scale
    ranks = g["ranks"]
    assert np.all(ranks[1:, :140] == ranks[0, :140])


def test_stop_spread_and_final_distance():
    g = _spread()
    iters = g["iters"]
    assert len(iters) == 21 and np.all(iters < 500)   # every run converged
    assert iters.max() - iters.min() >= 10             # the stop moves with rounding alone
    assert len(set(iters.tolist())) >= 5
    assert np.all(g["x_rel_diff_vs_base"] <= 2e-4)
    # tier B's stored complete run (another rounding of the same method)
    # stops inside the same range
    b = np.load(os.path.join(GOLDEN, "oracle_config2.npz"))
    assert iters.min() <= int(b["iters"]) <= iters.max()


def gpu_window():
    """The stop window and X tolerance for a complete run at this size that
    is not bitwise the oracle: the oracle's own stop range widened by half
    its width on each side, and twice the largest distance of a perturbed
    oracle run's X from the unperturbed one (any two runs, by the triangle
    inequality)."""
    g = _spread()
    lo, hi = int(g["iters"].min()), int(g["iters"].max())
    half = (hi - lo + 1) // 2
    return lo - half, hi + half, 2.0 * float(g["x_rel_diff_vs_base"].max())


def test_window_is_derived_from_the_spread():
    lo, hi, tol = gpu_window()
    assert lo < hi and 0 < tol < 1e-3
