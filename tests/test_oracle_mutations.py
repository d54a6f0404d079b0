"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in the oracle (on the CPU, by patching one of its
functions for the duration of the test) and checks that at least one of the
paper-derived pins then fails: the full-observation closed form, the kick
equivalence, or exact recovery of a Gaussian low-rank matrix.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.svt as osvt
import workload
from tests.test_oracle_svt import full_observation_closed_form


def _pins_pass() -> bool:
    try:
        # full observation, rectangular (catches transposes) and square
        for (m, n, sig) in [(30, 20, [400.0, 150.0, 60.0, 20.0]),
                            (12, 12, [500.0, 480.0, 30.0, 29.0, 5.3]),
                            (30, 20, [90.0, 50.0, 21.0])]:
            sig = np.array(sig)
            p, U, _, V = workload.full_observation(m, n, sig, seed=m + n)
            out = osvt.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta,
                                 p.eps, p.maxiter, p.incr)
            ref = full_observation_closed_form(sig, p.tau, p.delta, p.eps, p.maxiter)
            if out["k0"] != ref["k0"]:
                return False
            if out["iters"] != ref["iters"] or out["ranks"] != ref["ranks"]:
                return False
            Xref = (U * ref["x"]) @ V.T
            if np.linalg.norm(out["U"] @ out["V"].T - Xref) > 1e-10 * np.linalg.norm(Xref):
                return False
        # exact recovery on a small Gaussian instance
        n, r = 120, 4
        p = workload.gaussian_lowrank(n, n, r, 6 * workload.degrees_of_freedom(n, n, r),
                                      seed=0, tau=5.0 * n)
        out = osvt.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps,
                             300, p.incr)
        M = p.ML @ p.MR.T
        if out["status"] != "ok":
            return False
        if np.linalg.norm(out["U"] @ out["V"].T - M) > 1e-3 * np.linalg.norm(M):
            return False
        return True
    except (IndexError, ValueError, RuntimeError, FloatingPointError):
        return False


def test_unmodified_oracle_passes():
    assert _pins_pass()


def _transposed_sample(U, V, rows, cols):
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    return np.sum(U[cols] * V[rows], axis=1)


def _dropped_threshold_svd(A, *a, **k):
    U, s, V = _orig_jacobi(A, *a, **k)
    return U, s, V


_orig_jacobi = osvt.jacobi_svd
_orig_sample = osvt.sampled_entries
_orig_k0 = osvt.k0_kick


MUTATIONS = {
    # U and V exchanged in the sampled product
    "transposed_operand": ("sampled_entries", _transposed_sample),
    # X sampled with the wrong sign: flips the sign of the Y update
    "wrong_sign_update": ("sampled_entries",
                          lambda U, V, r, c: -_orig_sample(U, V, r, c)),
    # an off-by-one in the sampled term (a dropped rank-one term)
    "dropped_term": ("sampled_entries",
                     lambda U, V, r, c: _orig_sample(U[:, :-1], V[:, :-1], r, c)
                     if U.shape[1] > 0 else _orig_sample(U, V, r, c)),
    # k0 rounded down instead of up
    "k0_floor": ("k0_kick", lambda tau, delta, s1: max(1, math.floor(tau / (delta * s1)))),
    # k0 one too large
    "k0_plus_one": ("k0_kick", lambda tau, delta, s1: _orig_k0(tau, delta, s1) + 1),
    # singular values not sorted (largest last)
    "unsorted_svd": ("jacobi_svd",
                     lambda A, *a, **k: tuple(x[..., ::-1] if x.ndim > 1 else x[::-1]
                                              for x in _orig_jacobi(A, *a, **k))),
    # singular vectors of the transpose used on a rectangular matrix
    "swapped_singular_vectors": ("jacobi_svd",
                                 lambda A, *a, **k: (lambda U, s, V: (V, s, U))(
                                     *_orig_jacobi(A, *a, **k))),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(osvt, attr, fn)
    with np.errstate(all="ignore"):
        assert not _pins_pass(), f"planted mistake {name!r} was not caught"
