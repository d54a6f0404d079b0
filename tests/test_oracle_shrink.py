"""Pins for the oracle's singular value shrinkage operator D_tau.

Section 2.1: D_tau(Y) = U diag((sigma_i - tau)_+) V^T (eq. (2.2)), and
Theorem 2.1: D_tau(Y) is the unique minimiser of 1/2 ||X - Y||_F^2 + tau ||X||_*
(eq. (2.3)).  The proof exhibits the subgradient certificate
Y - D_tau(Y) = tau (U0 V0^T + W) with U0^T W = 0, W V0 = 0, ||W||_2 <= 1.
"""
import numpy as np
import pytest

from oracle import shrink


def _dense(Ur, w, Vr):
    return (Ur * w) @ Vr.T


def _nuclear(X):
    return np.linalg.svd(X, compute_uv=False).sum()  # LAPACK, independent of the oracle


@pytest.mark.parametrize("shape,tau", [((20, 14), 1.5), ((9, 17), 0.7), ((30, 30), 3.0)])
def test_subgradient_certificate(shape, tau):
    rng = np.random.default_rng(shape[0] * 7 + shape[1])
    Y = rng.standard_normal(shape) * 2.0
    Ur, w, Vr, _ = shrink(Y, tau)
    X = _dense(Ur, w, Vr)
    W = (Y - X) / tau - Ur @ Vr.T
    assert np.linalg.norm(Ur.T @ W) <= 1e-12
    assert np.linalg.norm(W @ Vr) <= 1e-12
    assert np.linalg.norm(W, 2) <= 1.0 + 1e-12


def test_prox_objective_not_beaten():
    rng = np.random.default_rng(11)
    Y = rng.standard_normal((15, 12)) * 3
    tau = 2.0
    Ur, w, Vr, _ = shrink(Y, tau)
    X = _dense(Ur, w, Vr)

    def h(Z):
        return 0.5 * np.linalg.norm(Z - Y) ** 2 + tau * _nuclear(Z)

    h0 = h(X)
    for scale in (1e-1, 1e-3, 1e-5):
        for _ in range(20):
            D = rng.standard_normal(Y.shape)
            assert h(X + scale * D) >= h0 - 1e-12 * abs(h0)


def test_diagonal_case_is_scalar_soft_threshold():
    d = np.array([5.0, -3.0, 0.5, -0.2, 2.0])
    Y = np.zeros((7, 5))
    Y[np.arange(5), np.arange(5)] = d
    tau = 1.0
    Ur, w, Vr, _ = shrink(Y, tau)
    expect = np.zeros_like(Y)
    expect[np.arange(5), np.arange(5)] = np.sign(d) * np.maximum(np.abs(d) - tau, 0)
    assert np.abs(_dense(Ur, w, Vr) - expect).max() <= 1e-14


def test_rank_one_closed_form():
    rng = np.random.default_rng(12)
    u = rng.standard_normal(10); u /= np.linalg.norm(u)
    v = rng.standard_normal(8); v /= np.linalg.norm(v)
    Y = 7.0 * np.outer(u, v)
    Ur, w, Vr, _ = shrink(Y, 2.5)
    assert Ur.shape[1] == 1 and abs(w[0] - 4.5) <= 1e-14 * 7
    assert np.abs(_dense(Ur, w, Vr) - 4.5 * np.outer(u, v)).max() <= 1e-14 * 7
    Ur, w, Vr, _ = shrink(Y, 7.5)
    assert Ur.shape[1] == 0


def test_identity_at_zero_threshold_and_zero_above_top():
    rng = np.random.default_rng(13)
    Y = rng.standard_normal((11, 6))
    Ur, w, Vr, s = shrink(Y, 0.0)
    assert np.abs(_dense(Ur, w, Vr) - Y).max() <= 1e-13
    Ur, w, Vr, _ = shrink(Y, s[0] * 1.0000001)
    assert Ur.shape[1] == 0


def test_homogeneity_and_orthogonal_invariance():
    rng = np.random.default_rng(14)
    Y = rng.standard_normal((13, 9)) * 2
    tau = 1.7
    X = _dense(*shrink(Y, tau)[:3])
    c = 3.25
    Xc = _dense(*shrink(c * Y, c * tau)[:3])
    assert np.abs(Xc - c * X).max() <= 1e-12 * np.abs(Xc).max()
    Q, _ = np.linalg.qr(rng.standard_normal((13, 13)))
    R, _ = np.linalg.qr(rng.standard_normal((9, 9)))
    Xq = _dense(*shrink(Q @ Y @ R, tau)[:3])
    assert np.abs(Xq - Q @ X @ R).max() <= 1e-12 * np.abs(X).max()
