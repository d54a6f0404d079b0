"""The matrix Dantzig selector by singular value thresholding: Section 3.3's
iteration for linear inequality constraints, specialised to matrix
completion (eq. (3.10)), in plain FP64.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may use this module.  It shares no code with the HIP
library.

Problem (Section 3.3, eq. (3.8) with A = P_Omega): minimise
tau ||X||_* + 1/2 ||X||_F^2 subject to |X_ij - B_ij| <= E_ij on Omega, where
B holds the (noisy) observations.  With a multiplier for each side of the
constraint, Y_+ and Y_- (nonnegative, supported on Omega), starting from
Y_+ = Y_- = 0, the iteration is

    X^k    = D_tau(Y_+^{k-1} - Y_-^{k-1})
    Y_+^k  = [Y_+^{k-1} + delta P_Omega( (B - X^k) - E)]_+
    Y_-^k  = [Y_-^{k-1} + delta P_Omega(-(B - X^k) - E)]_+

([.]_+ entrywise).  Readings taken where the paper leaves things open:

* the stop test: the relative constraint violation
  ||[ |P_Omega(X^k - B)| - E ]_+||_F / ||P_Omega B||_F <= eps, taken before the
  update as Algorithm 1 does; with E = 0 it is eq. (5.5).  stop="noisy"
  takes instead the data-consistency test of eq. (5.10),
  ||P_Omega(X^k - B)||_F^2 <= (1 + eps) |Omega| sigma^2 (Section 5.2.1's stop
  for noisy data); the recorded residual stays the relative violation;
* the kick (Section 5.1.3 carried over): while X = 0 the multipliers grow
  linearly, Y_+^k = k delta [B - E]_+ and Y_-^k = k delta [-B - E]_+, so
  Y_+ - Y_- = k delta S_E(B) with S_E the entrywise soft threshold; X^k stays
  0 up to k0 = ceil(tau / (delta ||S_E(P_Omega B)||_2)), and the iteration
  starts from Y_+^{k0}, Y_-^{k0}.  When S_E(B) = 0 (every |B_ij| <= E_ij)
  X = 0 is feasible and is returned at the first iteration;
* the s_k bookkeeping and the shrinkage are Algorithm 1's.
"""
from __future__ import annotations

import numpy as np

from .svt import _fro, jacobi_svd, k0_kick, sampled_entries


def soft_threshold(b, E):
    """S_E(b) = sign(b) max(|b| - E, 0), entrywise."""
    b = np.asarray(b, dtype=np.float64)
    return np.sign(b) * np.maximum(np.abs(b) - E, 0.0)


def _triplets_dense(m, n, rows, cols, y, r_prev, tau, incr, seed):
    Y = np.zeros((m, n))
    Y[rows, cols] = y
    U, s, V = jacobi_svd(Y)
    cap = min(m, n)
    s_k = min(r_prev + 1, cap)
    while s[s_k - 1] > tau and s_k < cap:
        s_k = min(s_k + incr, cap)
    return U, s, V, s_k


def _triplets_sparse(m, n, rows, cols, y, r_prev, tau, incr, seed):
    import scipy.sparse as sp

    from .krylov import top_triplets_sparse
    Y = sp.csr_matrix((y, (rows, cols)), shape=(m, n))
    cap = min(m, n)
    s_k = min(r_prev + 1, cap)
    while True:
        U, s, V = top_triplets_sparse(Y, s_k, seed)
        if s[s_k - 1] <= tau or s_k >= cap:
            return U, s, V, s_k
        s_k = min(s_k + incr, cap)


def svt_dantzig(m: int, n: int, rows, cols, b, E, tau: float, delta: float, eps: float,
                maxiter: int, incr: int, kick: bool = True, partial: str = "dense",
                seed: int = 0, keep_multipliers: bool = False, progress=None,
                stop: str = "violation", noise_sigma: float = 0.0):
    """The iteration above.  ``E``: a scalar or one tolerance per observed
    entry.  ``partial``: "dense" (full Jacobi SVD of the dense iterate, tier A)
    or "sparse" (the s_k largest triplets from the library partial SVD, tier
    C).  Returns iterations, k0, the histories of s_k, r_k and the relative
    violation, X as factors (U scaled by w, V) and, with keep_multipliers,
    the final Y_+ and Y_- (the ones X^k was formed from)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    b = np.asarray(b, dtype=np.float64)
    E = np.broadcast_to(np.asarray(E, dtype=np.float64), b.shape)
    if np.any(E < 0):
        raise ValueError("tolerances must be nonnegative")
    norm_b = _fro(b)
    triplets = _triplets_dense if partial == "dense" else _triplets_sparse
    yp = np.zeros_like(b)
    ym = np.zeros_like(b)
    k0 = 0
    sigma1 = None
    sb = soft_threshold(b, E)
    if kick:
        if np.any(sb != 0.0):
            if partial == "dense":
                S = np.zeros((m, n))
                S[rows, cols] = sb
                sigma1 = float(jacobi_svd(S)[1][0])
            else:
                sigma1 = float(_triplets_sparse(m, n, rows, cols, sb, 0, np.inf, incr, seed)[1][0])
            k0 = k0_kick(tau, delta, sigma1)
            yp = k0 * delta * np.maximum(b - E, 0.0)
            ym = k0 * delta * np.maximum(-b - E, 0.0)
        else:
            sigma1 = 0.0
    ranks, s_hist, res_hist = [], [], []
    r_prev = 0
    status = "not_converged"
    Uw = np.zeros((m, 0)); Vr = np.zeros((n, 0)); w = np.zeros(0)
    yp_used, ym_used = yp, ym
    k = 0
    for k in range(1, maxiter + 1):
        U, s, V, s_k = triplets(m, n, rows, cols, yp - ym, r_prev, tau, incr, seed + k)
        r_k = int(np.count_nonzero(s[:min(len(s), max(s_k, 1))] > tau))
        w = s[:r_k] - tau
        Uw = U[:, :r_k] * w
        Vr = V[:, :r_k]
        d = b - sampled_entries(Uw, Vr, rows, cols)
        viol = np.maximum(np.abs(d) - E, 0.0)
        res = _fro(viol) / norm_b
        ranks.append(r_k)
        s_hist.append(s_k)
        res_hist.append(res)
        if progress:
            progress(k, r_k, res)
        yp_used, ym_used = yp, ym
        if stop == "noisy":
            done = _fro(d) ** 2 <= (1.0 + eps) * b.shape[0] * noise_sigma ** 2
        else:
            done = res <= eps
        if done:
            status = "ok"
            break
        yp = np.maximum(yp + delta * (d - E), 0.0)
        ym = np.maximum(ym + delta * (-d - E), 0.0)
        r_prev = r_k
    out = dict(iters=k, k0=k0, sigma1=sigma1, ranks=ranks, s_hist=s_hist, residuals=res_hist,
               U=Uw, w=w, V=Vr, status=status, norm_b=norm_b)
    if keep_multipliers:
        out["yp"] = yp_used
        out["ym"] = ym_used
        out["yp_next"] = yp
        out["ym_next"] = ym
    return out


def dantzig_step(b, E, yp, ym, x, delta):
    """One multiplier update of the iteration with X's sampled entries x given:
    returns (Y_+, Y_-, squared violation of x)."""
    d = np.asarray(b, np.float64) - np.asarray(x, np.float64)
    viol = np.maximum(np.abs(d) - E, 0.0)
    return (np.maximum(yp + delta * (d - E), 0.0), np.maximum(ym + delta * (-d - E), 0.0),
            float(np.sum(viol * viol)))
