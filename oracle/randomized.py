"""Algorithm 1 with D_tau evaluated by a randomised SVD (the first direction
of Section 6), in plain FP64.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may use this module.  It shares no code with the HIP
library.

The s_k largest triplets of the sparse iterate Y (m x n) are approximated by
the randomised range finder with power iterations (Halko, Martinsson and
Tropp, 2011): with l = s + p columns (p the oversampling),

    Omega (n x l) Gaussian; Q = orth(Y Omega); then q times
    P = orth(Y^T Q), Q = orth(Y P); W = Y^T Q (n x l), so B = W^T = Q^T Y;
    W = Vw S Uw^T (a full SVD of the tall small matrix), so B = Uw S Vw^T;
    U = Q Uw, sigma = S, V = Vw.

orth() is any orthonormal basis of the columns' span (the subspaces, hence
the result, do not depend on which); here LAPACK's Householder QR.
Algorithm 1's repeat loop runs on top: s grows by ell (and l with it)
while the s-th approximate value is above tau.

The Gaussian test matrices come from a counter-based generator written out
from its published definition, so that another implementation can draw the
same numbers: SplitMix64's output function (Steele, Lea and Flood, 2014),
mix(z) = the 64-bit finaliser of z + 0x9E3779B97F4A7C15, keyed per matrix
by key = mix(seed xor mix(ctr)); entry i of a matrix uses a = mix(key + 2i)
and b = mix(key + 2i + 1) and the Box-Muller transform of the uniforms
u1 = (a >> 11 + 1) 2^-53 in (0, 1] and u2 = (b >> 11) 2^-53:
sqrt(-2 ln u1) cos(2 pi u2).  Matrices are filled column by column
(entry i = row + column * rows); ctr counts the matrices drawn in a solve.
"""
from __future__ import annotations

import math

import numpy as np

from .svt import _fro, jacobi_svd, k0_kick, sampled_entries

_MASK = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def splitmix_mix(z: int) -> int:
    """SplitMix64's output for state z (the state is advanced by the golden
    gamma first)."""
    z = (z + _GOLDEN) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def gaussian_matrix(rows: int, cols: int, seed: int, ctr: int) -> np.ndarray:
    """rows x cols standard normal draws of the generator above."""
    key = splitmix_mix((seed ^ splitmix_mix(ctr)) & _MASK)
    count = rows * cols
    i = np.arange(count, dtype=np.uint64)
    k = np.uint64(key)
    with np.errstate(over="ignore"):
        def mix(z):
            z = z + np.uint64(_GOLDEN)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            return z ^ (z >> np.uint64(31))
        a = mix(k + np.uint64(2) * i)
        b = mix(k + np.uint64(2) * i + np.uint64(1))
    u1 = ((a >> np.uint64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)
    u2 = (b >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
    return z.reshape(cols, rows).T.copy()


def _orth(Z):
    """Orthonormal columns spanning Z (Householder QR, LAPACK)."""
    Q, _ = np.linalg.qr(Z)
    return Q


def randomized_triplets(Ys, s: int, oversample: int, power: int, seed: int, ctr: int):
    """The approximate s largest triplets of the sparse Y (scipy CSR) as
    above; returns (U m x s, sigma[s], V n x s)."""
    m, n = Ys.shape
    cap = min(m, n)
    l = min(cap, s + oversample)
    Om = gaussian_matrix(n, l, seed, ctr)
    Q = _orth(np.asarray(Ys @ Om))
    for _ in range(power):
        P = _orth(np.asarray(Ys.T @ Q))
        Q = _orth(np.asarray(Ys @ P))
    W = np.asarray(Ys.T @ Q)                      # W = B^T, B = Q^T Y
    Vw, S, Uw = jacobi_svd(W)                     # W = Vw S Uw^T, so B = Uw S Vw^T
    U = Q @ Uw
    return U[:, :s], S[:s], Vw[:, :s]


def svt_randomized(m: int, n: int, rows, cols, vals, tau: float, delta: float, eps: float,
                   maxiter: int, incr: int, oversample: int = 10, power: int = 2, seed: int = 0,
                   kick: bool = True):
    """Algorithm 1 (Section 5.1.5) with the randomised triplets in place of
    the exact ones; the kick's ||P_Omega M||_2 is taken exactly (Jacobi on
    the dense matrix for small sizes, the same randomised route otherwise is
    not used: the kick needs one exact value).  ctr advances by one per test
    matrix drawn (the kick draws none)."""
    import scipy.sparse as sp
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    norm_pm = _fro(vals)
    cap = min(m, n)
    y = np.zeros_like(vals)
    k0 = 0
    sigma1 = None
    if kick:
        PM = np.zeros((m, n))
        PM[rows, cols] = vals
        sigma1 = float(jacobi_svd(PM)[1][0])
        k0 = k0_kick(tau, delta, sigma1)
        y = k0 * delta * vals
    ranks, s_hist, res_hist = [], [], []
    r_prev = 0
    status = "not_converged"
    Uw = np.zeros((m, 0)); Vr = np.zeros((n, 0)); w = np.zeros(0)
    ctr = 0
    k = 0
    for k in range(1, maxiter + 1):
        Ys = sp.csr_matrix((y, (rows, cols)), shape=(m, n))
        s_k = min(r_prev + 1, cap)
        while True:
            U, S, V = randomized_triplets(Ys, s_k, oversample, power, seed, ctr)
            ctr += 1
            if S[s_k - 1] <= tau or s_k >= cap:
                break
            s_k = min(s_k + incr, cap)
        r_k = int(np.count_nonzero(S > tau))
        w = S[:r_k] - tau
        Uw = U[:, :r_k] * w
        Vr = V[:, :r_k]
        e = vals - sampled_entries(Uw, Vr, rows, cols)
        res = _fro(e) / norm_pm
        ranks.append(r_k)
        s_hist.append(s_k)
        res_hist.append(res)
        if res <= eps:
            status = "ok"
            break
        y = y + delta * e
        r_prev = r_k
    return dict(iters=k, k0=k0, sigma1=sigma1, ranks=ranks, s_hist=s_hist, residuals=res_hist,
                U=Uw, w=w, V=Vr, status=status)
