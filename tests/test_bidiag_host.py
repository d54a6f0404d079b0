"""Host bidiagonal SVD (the Ritz step of the bidiagonalisation, Section 5.1.1)
checked against LAPACK's SVD through numpy on small and large B_k.

The library's bidiag.cpp is compiled here with g++ together with a small
stdin/stdout driver; nothing runs on a GPU.  Checked: singular values,
|last row of P| (the residual bounds' factor) for well separated values,
the first nvec right vectors up to sign, P = B Q / sigma, and the
orthonormality of Q -- including a k = 320, nvec = 58 case whose vectors
take the threaded path, a matrix with a zero diagonal entry, one that splits
at a zero superdiagonal, and k = 1.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0810_3286_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("bidiag") / "bidiag_driver")
    subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", f"-I{CSRC}",
                    os.path.join(ROOT, "tests", "bidiag_driver.cpp"), os.path.join(CSRC, "bidiag.cpp"),
                    "-o", exe], check=True)
    return exe


def run(exe, d, e, nvec):
    k = len(d)
    text = f"{k} {nvec}\n" + "\n".join(repr(float(x)) for x in list(d) + list(e)) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout.split()
    assert out[0] != "FAIL"
    v = np.array([float(x) for x in out])
    sigma, plast = v[:k], v[k:2 * k]
    Q = v[2 * k:2 * k + k * nvec].reshape(nvec, k).T
    P = v[2 * k + k * nvec:].reshape(nvec, k).T
    return sigma, plast, Q, P


def dense(d, e):
    k = len(d)
    B = np.diag(np.asarray(d, dtype=np.float64))
    if k > 1:
        B += np.diag(np.asarray(e, dtype=np.float64), 1)
    return B


def lanczos_like(k, seed, top=10):
    """A bidiagonal with the spread of a Lanczos B_k of a low-rank iterate:
    a few large diagonal entries over a bulk of comparable ones."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.5, 2.0, k) * 1e5
    e = rng.uniform(0.5, 2.0, k - 1) * 5e4
    d[:top] *= 20.0
    return d, e


def check(exe, d, e, nvec, sep_tol=1e-3):
    B = dense(d, e)
    k = B.shape[0]
    U, s, Vt = np.linalg.svd(B)
    sigma, plast, Q, P = run(exe, d, e, nvec)
    s1 = max(s[0], 1e-300)
    assert np.all(np.diff(sigma) <= 0.0)
    np.testing.assert_allclose(sigma, s, rtol=0, atol=1e-13 * s1)
    # vectors and last-row entries are unique only for separated values
    gaps = np.full(k, np.inf)
    if k > 1:
        g = np.abs(np.diff(s))
        gaps[:-1] = g
        gaps[1:] = np.minimum(gaps[1:], g)
    sep = gaps > sep_tol * s1
    np.testing.assert_allclose(np.abs(plast[sep]), np.abs(U[-1, sep]), rtol=0, atol=1e-9)
    for i in range(nvec):
        if sep[i]:
            v = Vt[i]
            sg = np.sign(v @ Q[:, i])
            np.testing.assert_allclose(Q[:, i], sg * v, rtol=0, atol=1e-9)
    np.testing.assert_allclose(Q.T @ Q, np.eye(nvec), rtol=0, atol=1e-12)
    for i in range(nvec):
        if sigma[i] > 1e-12 * s1:
            np.testing.assert_allclose(B @ Q[:, i], sigma[i] * P[:, i], rtol=0, atol=1e-12 * s1)


@pytest.mark.parametrize("k,nvec,seed", [(5, 5, 0), (55, 11, 1), (150, 20, 2), (320, 58, 3)])
def test_bidiag_matches_lapack(driver, k, nvec, seed):
    d, e = lanczos_like(k, seed)
    check(driver, d, e, nvec)


def test_bidiag_single(driver):
    sigma, plast, Q, P = run(driver, [-3.0], [], 1)
    assert sigma[0] == 3.0 and abs(plast[0]) == 1.0
    assert abs(Q[0, 0]) == 1.0 and abs(P[0, 0]) == 1.0


def test_bidiag_zero_diagonal_and_split(driver):
    d, e = lanczos_like(40, 4, top=3)
    d[17] = 0.0          # a zero singular value: chased out along its row
    d[39] = 0.0          # last diagonal zero: chased up its column
    e[25] = 0.0          # splits into two blocks
    check(driver, d, e, 12)


def gkl_coefficients(A, k, seed):
    """alpha, beta of k steps of the Golub-Kahan bidiagonalisation of A
    (Section 5.1.1's partial SVD) with full reorthogonalisation, in numpy:
    the B_k of an actual low-rank-plus-noise matrix."""
    rng = np.random.default_rng(seed)
    m, n = A.shape
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    U, V = np.zeros((m, k)), np.zeros((n, k))
    alpha, beta = np.zeros(k), np.zeros(k)
    u_prev, b = np.zeros(m), 0.0
    for j in range(k):
        V[:, j] = v
        u = A @ v - b * u_prev
        u -= U[:, :j] @ (U[:, :j].T @ u)
        alpha[j] = np.linalg.norm(u)
        u /= alpha[j]
        U[:, j] = u
        w = A.T @ u - alpha[j] * v
        w -= V[:, :j + 1] @ (V[:, :j + 1].T @ w)
        b = np.linalg.norm(w)
        beta[j] = b
        v, u_prev = w / b, u
    # B_k upper bidiagonal: diagonal alpha, superdiagonal beta_2 .. beta_k
    return alpha, beta[:-1]


@pytest.mark.parametrize("k,rank,seed", [(60, 10, 5), (200, 50, 6)])
def test_bidiag_lanczos_matrix(driver, k, rank, seed):
    rng = np.random.default_rng(seed)
    m, n = 400, 300
    A = rng.standard_normal((m, rank)) @ rng.standard_normal((rank, n)) * 10.0 + 0.1 * rng.standard_normal((m, n))
    d, e = gkl_coefficients(A, k, seed)
    check(driver, d, e, min(rank + 1, k))


def test_bidiag_graded_and_clustered(driver):
    rng = np.random.default_rng(7)
    k = 120
    d = 1e6 * 0.8 ** np.arange(k)        # graded over many orders of magnitude
    e = d[:-1] * rng.uniform(0.01, 0.5, k - 1)
    check(driver, d, e, 20)
    d = np.full(k, 3.0) + 1e-10 * rng.standard_normal(k)   # one tight cluster
    e = 1e-3 * rng.uniform(0.5, 1.0, k - 1)
    check(driver, d, e, 8)
