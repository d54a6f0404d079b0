"""Host dense kernels of the randomised partial SVD (Section 6) checked
against LAPACK through numpy: the orthonormal basis spans the input's
columns and is orthonormal; the one-sided Jacobi SVD of a tall matrix
reconstructs it, has orthonormal factors and LAPACK's singular values
(well and badly conditioned cases, a rank-deficient one, one column).
dense_host.cpp is compiled here with g++ with a stdin/stdout driver;
nothing runs on a GPU."""
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
    exe = str(tmp_path_factory.mktemp("dense") / "dense_driver")
    subprocess.run([gxx, "-O2", "-std=c++17", f"-I{CSRC}", os.path.join(ROOT, "tests", "dense_driver.cpp"),
                    os.path.join(CSRC, "dense_host.cpp"), "-o", exe], check=True)
    return exe


def run(exe, op, A):
    rows, cols = A.shape
    text = f"{op} {rows} {cols}\n" + "\n".join(repr(float(x)) for x in A.T.ravel()) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout.split()
    assert out[0] != "FAIL"
    return np.array([float(x) for x in out])


@pytest.mark.parametrize("rows,cols,seed", [(50, 7, 0), (300, 20, 1), (1000, 3, 2)])
def test_orth_columns(driver, rows, cols, seed):
    A = np.random.default_rng(seed).standard_normal((rows, cols)) * np.logspace(0, 6, cols)
    Q = run(driver, 0, A).reshape(cols, rows).T
    assert np.linalg.norm(Q.T @ Q - np.eye(cols)) <= 1e-13 * cols
    # the same span: A = Q (Q^T A)
    assert np.linalg.norm(A - Q @ (Q.T @ A)) <= 1e-12 * np.linalg.norm(A)
    # Gram-Schmidt keeps the leading columns' span: Q^T A upper triangular
    R = Q.T @ A
    assert np.linalg.norm(np.tril(R, -1)) <= 1e-12 * np.linalg.norm(R)


def test_orth_columns_rank_deficient(driver):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 3))
    A = np.hstack([A, A[:, :1] * 2.0 + A[:, 1:2]])   # the 4th column lies in the span
    Q = run(driver, 0, A).reshape(4, 40).T
    assert np.linalg.norm(Q[:, 3]) == 0.0
    assert np.linalg.norm(Q[:, :3].T @ Q[:, :3] - np.eye(3)) <= 1e-13


@pytest.mark.parametrize("rows,cols,seed,spread", [(60, 8, 0, 1.0), (500, 25, 1, 1e6), (2000, 12, 2, 1e3),
                                                    (30, 1, 3, 1.0)])
def test_jacobi_svd_tall(driver, rows, cols, seed, spread):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((rows, cols)) @ np.diag(np.logspace(0, np.log10(spread), cols)) @ \
        np.linalg.qr(rng.standard_normal((cols, cols)))[0]
    v = run(driver, 1, A)
    s = v[:cols]
    V = v[cols:cols + rows * cols].reshape(cols, rows).T
    U = v[cols + rows * cols:].reshape(cols, cols).T
    ref = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(s, ref, rtol=1e-13, atol=1e-14 * ref[0])
    assert np.all(np.diff(s) <= 0)
    assert np.linalg.norm(V.T @ V - np.eye(cols)) <= 1e-12 * cols
    assert np.linalg.norm(U.T @ U - np.eye(cols)) <= 1e-13 * cols
    assert np.linalg.norm(A - (V * s) @ U.T) <= 1e-13 * np.linalg.norm(A)


def test_jacobi_svd_rank_deficient(driver):
    rng = np.random.default_rng(5)
    B = rng.standard_normal((80, 3))
    A = np.hstack([B, B @ rng.standard_normal((3, 2))])
    v = run(driver, 1, A)
    s = v[:5]
    V = v[5:5 + 80 * 5].reshape(5, 80).T
    U = v[5 + 80 * 5:].reshape(5, 5).T
    np.testing.assert_allclose(s[:3], np.linalg.svd(A, compute_uv=False)[:3], rtol=1e-12)
    assert np.all(s[3:] <= 1e-12 * s[0])
    assert np.linalg.norm(A - (V * s) @ U.T) <= 1e-12 * np.linalg.norm(A)
