"""SVT for a general linear operator: Uzawa's iteration of Section 3.1,
eq. (3.3), in plain FP64 with a dense iterate and a full Jacobi SVD.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may use this module.  It shares no code with the HIP
library.

The operator A maps n1 x n2 matrices to R^p through entries on a support
set S (positions (srows[s], scols[s]), s = 0..|S|-1): A(X) = G x_S, where x_S
holds X's entries on S and G is a sparse p x |S| matrix (measurement i is
sum_s G[i, s] X[srows[s], scols[s]]).  Its adjoint puts G^T y on S:
A*(y) = sum_s (G^T y)_s e_{srows[s]} e_{scols[s]}^T.  Starting from y = 0,

    X^k = D_tau(A*(y^{k-1})),     y^k = y^{k-1} + delta (b - A(X^k)).

Completion is the case G = identity on S = Omega (A* A = P_Omega), where
this is Algorithm 1's iteration with Y^k = A*(y^k) (Section 3.1).  Readings
carried over from Algorithm 1: the kick (while X = 0, y^k = k delta b, so X
stays 0 up to k0 = ceil(tau / (delta ||A*(b)||_2)), eq. (5.3) with A*(b) in
place of P_Omega M); the stop test ||b - A(X^k)|| / ||b|| <= eps (eq. (5.5)
with the measurements in place of the samples); Algorithm 1's s_k
bookkeeping.
"""
from __future__ import annotations

import numpy as np

from .svt import _fro, jacobi_svd, k0_kick, sampled_entries


def adjoint(m: int, n: int, srows, scols, G, y):
    """A*(y) as a dense m x n matrix."""
    Y = np.zeros((m, n))
    np.add.at(Y, (np.asarray(srows), np.asarray(scols)), G.T @ y)
    return Y


def svt_general(m: int, n: int, srows, scols, G, b, tau: float, delta: float, eps: float,
                maxiter: int, incr: int, kick: bool = True):
    """Eq. (3.3) as above.  G: scipy.sparse p x |S|; b: p measurements.
    Returns iterations, k0, histories of s_k, r_k and ||b - A(X^k)|| / ||b||,
    and X as factors (U scaled by w, V)."""
    srows = np.asarray(srows, dtype=np.int64)
    scols = np.asarray(scols, dtype=np.int64)
    b = np.asarray(b, dtype=np.float64)
    norm_b = _fro(b)
    cap = min(m, n)
    y = np.zeros_like(b)
    k0 = 0
    sigma1 = None
    if kick:
        sigma1 = float(jacobi_svd(adjoint(m, n, srows, scols, G, b))[1][0])
        k0 = k0_kick(tau, delta, sigma1)
        y = k0 * delta * b
    ranks, s_hist, res_hist = [], [], []
    r_prev = 0
    status = "not_converged"
    Uw = np.zeros((m, 0)); Vr = np.zeros((n, 0)); w = np.zeros(0)
    k = 0
    for k in range(1, maxiter + 1):
        U, s, V = jacobi_svd(adjoint(m, n, srows, scols, G, y))
        s_k = min(r_prev + 1, cap)
        while s[s_k - 1] > tau and s_k < cap:
            s_k = min(s_k + incr, cap)
        r_k = int(np.count_nonzero(s > tau))
        w = s[:r_k] - tau
        Uw = U[:, :r_k] * w
        Vr = V[:, :r_k]
        resid = b - G @ sampled_entries(Uw, Vr, srows, scols)
        res = _fro(resid) / norm_b
        ranks.append(r_k)
        s_hist.append(s_k)
        res_hist.append(res)
        if res <= eps:
            status = "ok"
            break
        y = y + delta * resid
        r_prev = r_k
    return dict(iters=k, k0=k0, sigma1=sigma1, ranks=ranks, s_hist=s_hist, residuals=res_hist,
                U=Uw, w=w, V=Vr, status=status, y=y)
