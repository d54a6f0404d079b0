"""Pins for the oracle's one-sided Jacobi SVD.

The Jacobi SVD is checked against things other than itself: LAPACK's SVD
(numpy.linalg.svd, an independent library routine), the closed form of the
2 x 2 singular values, exact reconstruction and orthogonality, and special
matrices whose singular values are known by construction.
"""
import math

import numpy as np
import pytest

from oracle import jacobi_svd


def _check_svd(A, U, s, V, tol=1e-13):
    m, n = A.shape
    k = min(m, n)
    assert U.shape == (m, k) and V.shape == (n, k) and s.shape == (k,)
    scale = max(np.linalg.norm(A, 2), 1e-300)
    # reconstruction
    assert np.linalg.norm(A - (U * s) @ V.T) <= tol * 10 * scale * math.sqrt(k)
    # descending and nonnegative
    assert np.all(np.diff(s) <= 0) and np.all(s >= 0)
    # orthonormal vectors for the nonzero singular values
    nz = s > 1e-10 * scale
    assert np.linalg.norm(U[:, nz].T @ U[:, nz] - np.eye(nz.sum())) <= 1e-12
    assert np.linalg.norm(V.T @ V - np.eye(k)) <= 1e-12


@pytest.mark.parametrize("shape", [(60, 40), (40, 60), (25, 25), (7, 1), (1, 9), (1, 1)])
def test_against_lapack_random(shape):
    rng = np.random.default_rng(hash(shape) % 1000)
    A = rng.standard_normal(shape)
    U, s, V = jacobi_svd(A)
    ref = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(s - ref)) <= 1e-13 * ref[0]
    _check_svd(A, U, s, V)


def test_rank_deficient():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 5)) @ rng.standard_normal((5, 20))
    U, s, V = jacobi_svd(A)
    ref = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(s - ref)) <= 1e-13 * ref[0]
    assert np.all(s[5:] <= 1e-12 * s[0])
    _check_svd(A, U, s, V)


def test_repeated_singular_values():
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    R, _ = np.linalg.qr(rng.standard_normal((9, 9)))
    sig = np.array([3.0, 3.0, 3.0, 1.0, 1.0, 0.5, 0.5, 0.5, 0.25])
    A = Q[:, :9] @ np.diag(sig) @ R.T
    U, s, V = jacobi_svd(A)
    assert np.max(np.abs(s - sig)) <= 1e-14 * 3
    _check_svd(A, U, s, V)


def test_graded_matrix():
    # singular values spread over ten decades: one-sided Jacobi computes the
    # small ones to high relative accuracy on a column-graded matrix
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((20, 20)))
    sig = np.logspace(0, -10, 15)
    A = Q[:, :15] * sig
    U, s, V = jacobi_svd(A)
    assert np.max(np.abs(s - sig) / sig) <= 1e-12
    _check_svd(A, U, s, V)


@pytest.mark.parametrize("a,b,c,d", [(1.0, 2.0, 3.0, 4.0), (2.0, 0.0, 0.0, -3.0),
                                      (1e-3, 5.0, -7.0, 0.5), (1.0, 1.0, 1.0, 1.0)])
def test_two_by_two_closed_form(a, b, c, d):
    # For [[a, b], [c, d]]: sigma^2 are the roots of x^2 - F x + D^2 with
    # F = a^2+b^2+c^2+d^2 and D = ad - bc.
    A = np.array([[a, b], [c, d]])
    F = a * a + b * b + c * c + d * d
    D = a * d - b * c
    disc = math.sqrt(max(F * F - 4 * D * D, 0.0))
    s1 = math.sqrt((F + disc) / 2)
    s2 = abs(D) / s1
    _, s, _ = jacobi_svd(A)
    assert abs(s[0] - s1) <= 1e-14 * s1
    assert abs(s[1] - s2) <= 1e-14 * s1


def test_zero_matrix():
    A = np.zeros((5, 3))
    U, s, V = jacobi_svd(A)
    assert np.all(s == 0)
    assert np.linalg.norm(V.T @ V - np.eye(3)) == 0


def test_orthogonal_matrix_has_unit_singular_values():
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((16, 16)))
    _, s, _ = jacobi_svd(Q)
    assert np.max(np.abs(s - 1)) <= 1e-14
