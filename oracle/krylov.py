"""Tier C of the CPU oracle: Algorithm 1 on a sparse iterate, each partial
SVD taken by a library routine, as the paper does.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may use this module.  It shares no code with the HIP
library.

Why a third tier.  Tier A (``svt_dense``) takes a full Jacobi SVD of a dense
iterate and tier B (``svt_sparse``) the eigendecomposition of the dense Gram
matrix; at 30000 x 30000 the first needs 7.2 GB per iterate and the second
about 12 minutes per iteration.  Algorithm 1 (Section 5.1.5) never asks for
more than the s_k largest singular triplets of the iterate, and the paper
computes them with a library (PROPACK, Section 5.1.1).  This tier does the
same with the partial SVD of SciPy (``scipy.sparse.linalg.svds`` with
ARPACK: implicitly restarted Lanczos on the Gram operator of the smaller
side, stopped at machine precision, followed by a Rayleigh-Ritz SVD of
Y V with LAPACK).  It shares neither code nor method with the product's
bidiagonalisation.

Algorithm 1's inner repeat loop is taken as printed: with s = r_{k-1} + 1,
compute the s largest triplets; while the s-th value is above tau, add ell
to s and compute them again.  The recorded s_k is the count of the last
computation, as in the other tiers.
"""
from __future__ import annotations

import numpy as np

from .svt import _fro, jacobi_svd, k0_kick, sampled_entries


def top_triplets_sparse(Yr, s: int, seed: int = 0):
    """The s largest singular triplets of a sparse Y (Algorithm 1's
    [U, Sigma, V]_s), descending: (U m x s, sigma[s], V n x s).

    SciPy's ``svds`` (ARPACK, tol = 0: machine precision) with a seeded start
    vector.  ARPACK needs s < min(m, n); at or above that (tiny matrices
    only) the full one-sided Jacobi SVD of the dense Y is taken instead.
    """
    from scipy.sparse.linalg import svds
    m, n = Yr.shape
    if s >= min(m, n) - 1:
        U, S, V = jacobi_svd(Yr.toarray())
        return U[:, :s], S[:s], V[:, :s]
    v0 = np.random.default_rng(seed).standard_normal(min(m, n))
    u, S, vt = svds(Yr, k=s, solver="arpack", tol=0, v0=v0)
    order = np.argsort(S)[::-1]
    return u[:, order], S[order], vt[order].T


def svt_krylov(m: int, n: int, rows, cols, vals, tau: float, delta: float,
               eps: float, maxiter: int, incr: int, kick: bool = True,
               seed: int = 0, progress=None, keep_iterates_at=(),
               max_seconds: float | None = None):
    """Algorithm 1 (Section 5.1.5), tier C: sparse Y, the s_k largest
    triplets by a library partial SVD (``top_triplets_sparse``).

    Steps and order as ``svt_dense``: the kick of eq. (5.3) (||P_Omega M||_2
    from the same routine), then for k = 1..maxiter the repeat loop over s_k,
    r_k = max{j : sigma_j > tau}, X^k as factors, the stop test of eq. (5.5),
    Y += delta P_Omega(M - X^k) (eq. (2.7)).  ``keep_iterates_at``: loop
    counters whose X^k (U scaled by w, w, V) is returned in ``snapshots``.
    ``max_seconds``: end the loop (status "time_limit") once it has run that
    long, for bounded timings.  ``y_last``: the iterate after the last update
    (in the input order of the samples), the Y that the next iteration would
    take its triplets of.
    """
    import time

    import scipy.sparse as sp
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    norm_pm = _fro(vals)
    cap = min(m, n)
    order = np.lexsort((cols, rows))
    rs, cs = rows[order], cols[order]

    def as_sparse(y):
        return sp.csr_matrix((y[order], (rs, cs)), shape=(m, n))

    sigma1 = None
    y = np.zeros(vals.shape[0])
    k0 = 0
    if kick:
        sigma1 = float(top_triplets_sparse(as_sparse(vals), 1, seed)[1][0])
        k0 = k0_kick(tau, delta, sigma1)
        y = k0 * delta * vals
    ranks, s_hist, res_hist, seconds = [], [], [], []
    snapshots = {}
    r_prev = 0
    status = "not_converged"
    Uw = np.zeros((m, 0)); Vr = np.zeros((n, 0)); w = np.zeros(0)
    k = 0
    t_loop = time.perf_counter()
    for k in range(1, maxiter + 1):
        t_it = time.perf_counter()
        Y = as_sparse(y)
        s_k = min(r_prev + 1, cap)
        while True:
            U, S, V = top_triplets_sparse(Y, s_k, seed + k)
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
        seconds.append(time.perf_counter() - t_it)
        if k in keep_iterates_at:
            snapshots[k] = (Uw.copy(), w.copy(), Vr.copy())
        if progress:
            progress(k, r_k, res)
        if res <= eps:
            status = "ok"
            break
        y = y + delta * e
        r_prev = r_k
        if max_seconds is not None and time.perf_counter() - t_loop >= max_seconds:
            status = "time_limit"
            break
    return dict(iters=k, k0=k0, sigma1=sigma1, ranks=ranks, s_hist=s_hist,
                residuals=res_hist, U=Uw, w=w, V=Vr, status=status, norm_pm=norm_pm,
                seconds=seconds, snapshots=snapshots, y_last=y)
