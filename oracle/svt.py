"""Plain FP64 CPU implementation of the SVT iteration (tier A: dense iterate).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may use this module.  It shares no code with the HIP library.

Notation follows the paper: the unknown matrix is n1 x n2 (here m x n), the
observed set is Omega, P_Omega keeps the entries in Omega and zeroes the rest,
D_tau is the singular value shrinkage operator (Section 2.1, eq. (2.2)).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

# Jacobi settings: pair-orthogonality threshold and sweep cap.
JACOBI_TOL = 1e-15
JACOBI_MAX_SWEEPS = 60


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_jacobi_svd.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp,
                                          ctypes.c_double, ctypes.c_int]
        lib.oracle_jacobi_svd.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def jacobi_svd(A: np.ndarray, tol: float = JACOBI_TOL,
               max_sweeps: int = JACOBI_MAX_SWEEPS):
    """Full SVD A = U diag(s) V^T by one-sided Jacobi (see ``jacobi.c``).

    Returns (U, s, V) with k = min(m, n) columns, s descending.  A wide matrix
    is handled through its transpose.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        Vt, s, Ut = jacobi_svd(A.T, tol, max_sweeps)
        return Ut, s, Vt
    work = np.array(A, dtype=np.float64, order="F", copy=True)
    V = np.zeros((n, n), dtype=np.float64, order="F")
    s = np.zeros(n, dtype=np.float64)
    sweeps = _load().oracle_jacobi_svd(m, n, _ptr(work), _ptr(V), _ptr(s),
                                       tol, max_sweeps)
    if sweeps < 0:
        raise RuntimeError(f"one-sided Jacobi did not converge (code {sweeps})")
    return work, s, V


def shrink(Y: np.ndarray, tau: float):
    """Singular value shrinkage D_tau(Y) (Section 2.1, eq. (2.2)).

    D_tau(Y) = U diag((sigma_i - tau)_+) V^T on the SVD of Y.  Returns
    (U_r, w, V_r, sigma): the r singular vectors with sigma_i > tau, the weights
    w_i = sigma_i - tau, and all singular values of Y, so that
    D_tau(Y) = U_r diag(w) V_r^T.
    """
    U, s, V = jacobi_svd(Y)
    r = int(np.count_nonzero(s > tau))
    return U[:, :r], s[:r] - tau, V[:, :r], s


def top_triplets_dense(Y: np.ndarray, count: int):
    """The ``count`` largest singular triplets of a dense matrix (full SVD)."""
    U, s, V = jacobi_svd(Y)
    return U[:, :count], s[:count], V[:, :count]


def k0_kick(tau: float, delta: float, sigma1: float) -> int:
    """k0 with tau / (delta ||P_Omega M||_2) in (k0 - 1, k0]  (Section 5.1.3, eq. (5.3)).

    Since Y^0 = 0, X^k = 0 and Y^k = k delta P_Omega(M) for k <= k0, so the
    iteration may start from Y^{k0}.
    """
    q = tau / (delta * sigma1)
    return max(1, int(math.ceil(q)))


def apply_sparse(m: int, n: int, rows, cols, yvals, x, trans: bool = False):
    """Y x (or Y^T x) for Y supported on Omega (Section 2.2, sparsity property).

    Plain definition: (Y x)_i = sum over (i, j) in Omega of Y_ij x_j.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    yvals = np.asarray(yvals, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    if not trans:
        out = np.zeros(m, dtype=np.float64)
        np.add.at(out, rows, yvals * x[cols])
    else:
        out = np.zeros(n, dtype=np.float64)
        np.add.at(out, cols, yvals * x[rows])
    return out


def sampled_entries(U: np.ndarray, V: np.ndarray, rows, cols):
    """X_ij = sum_l U_il V_jl for (i, j) in Omega: P_Omega of a factored X."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    out = np.zeros(rows.shape[0], dtype=np.float64)
    for l in range(U.shape[1]):
        out += U[rows, l] * V[cols, l]
    return out


def _fro(vec) -> float:
    """Euclidean norm with an exactly rounded sum of squares (math.fsum)."""
    v = np.asarray(vec, dtype=np.float64)
    return math.sqrt(math.fsum((v * v).tolist()))


def svt_dense(m: int, n: int, rows, cols, vals, tau: float, delta: float,
              eps: float, maxiter: int, incr: int, kick: bool = True,
              k0: int | None = None, stop: str = "relres", noise_sigma: float = 0.0,
              keep_iterates: bool = False, y0=None):
    """Algorithm 1 (Section 5.1.5) with a dense iterate and a full Jacobi SVD.

    Steps, in the paper's order:
      * Y^0 = k0 delta P_Omega(M), k0 from eq. (5.3) (skipped when kick=False:
        then Y^0 = 0 and k0 = 0);
      * for k = 1..k_max:
          - s_k = r_{k-1} + 1, and s_k grows by ell while the s_k-th singular
            value of Y^{k-1} is above tau (Section 5.1.1).  With the full SVD at
            hand this only records s_k; X^k does not depend on it;
          - r_k = max{j : sigma_j > tau};
          - X^k = sum_{j <= r_k} (sigma_j - tau) u_j v_j^T;
          - stop when ||P_Omega(X^k - M)||_F / ||P_Omega M||_F <= eps
            (eq. (5.5)); with stop="noisy", when
            ||P_Omega(X^k - B)||_F^2 <= (1 + eps) |Omega| sigma^2 (eq. (5.10));
          - Y^k = Y^{k-1} + delta P_Omega(M - X^k)  (eq. (2.7)).
    Returns a dict with the iteration count (Algorithm 1's loop counter at the
    break, not counting the k0 skipped steps), k0, and the histories of s_k,
    r_k and the relative residual, and X^opt as factors (U scaled by the
    weights sigma_j - tau, and V).
    ``y0`` (values on Omega, in the input order): start from Y^0 = y0 instead
    (no kick: a warm start); ``y_last`` in the result is the last iterate
    with the final update of eq. (2.7) applied, Y^{k} = Y^{k-1} + delta
    P_Omega(M - X^k), the state a following warm start continues from.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    nnz = rows.shape[0]
    norm_pm = _fro(vals)
    cap = min(m, n)

    Y = np.zeros((m, n), dtype=np.float64)
    sigma1 = None
    if y0 is not None:
        Y[rows, cols] = np.asarray(y0, dtype=np.float64)
        kick, k0 = False, 0
    if kick:
        PM = np.zeros((m, n), dtype=np.float64)
        PM[rows, cols] = vals
        sigma1 = float(jacobi_svd(PM)[1][0])
        if k0 is None:
            k0 = k0_kick(tau, delta, sigma1)
        Y[rows, cols] = k0 * delta * vals
    elif y0 is None:
        k0 = 0

    ranks, s_hist, res_hist = [], [], []
    iterates = []
    y_hist = [Y[rows, cols].copy()] if keep_iterates else None
    r_prev = 0
    status = "not_converged"
    Uw = np.zeros((m, 0))
    Vr = np.zeros((n, 0))
    w = np.zeros(0)
    k = 0
    for k in range(1, maxiter + 1):
        U, s, V = jacobi_svd(Y)
        s_k = min(r_prev + 1, cap)
        while s[s_k - 1] > tau and s_k < cap:
            s_k = min(s_k + incr, cap)
        r_k = int(np.count_nonzero(s > tau))
        w = s[:r_k] - tau
        Uw = U[:, :r_k] * w
        Vr = V[:, :r_k]
        e = vals - sampled_entries(Uw, Vr, rows, cols)
        res = _fro(e) / norm_pm
        ranks.append(r_k)
        s_hist.append(s_k)
        res_hist.append(res)
        if keep_iterates:
            iterates.append((Uw.copy(), Vr.copy()))
        if stop == "noisy":
            done = _fro(e) ** 2 <= (1.0 + eps) * nnz * noise_sigma ** 2
        else:
            done = res <= eps
        if done:
            status = "ok"
            break
        Y[rows, cols] += delta * e
        if keep_iterates:
            y_hist.append(Y[rows, cols].copy())
        r_prev = r_k
    y_last = Y[rows, cols] + (delta * e if status == "ok" else 0.0)
    out = dict(iters=k, k0=k0, sigma1=sigma1, ranks=ranks, s_hist=s_hist,
               residuals=res_hist, U=Uw, w=w, V=Vr, status=status,
               norm_pm=norm_pm, y_last=y_last)
    if keep_iterates:
        out["iterates"] = iterates
        out["y_hist"] = y_hist
        out["Y"] = Y
    return out


def svt_continuation(m: int, n: int, rows, cols, vals, taus, delta: float, eps: float,
                     maxiter: int, incr: int):
    """tau continuation with warm starts (Section 6): Algorithm 1 for each
    tau_i of an increasing schedule, the first from the kick, each later one
    from the previous one's last iterate Y (``svt_dense``'s y0).  The dual
    iterate is carried rather than a primal guess, so Y stays supported on
    Omega.  Returns the list of the stages' results."""
    stages = []
    y = None
    for t in taus:
        out = svt_dense(m, n, rows, cols, vals, float(t), delta, eps, maxiter, incr, y0=y)
        stages.append(out)
        y = out["y_last"]
    return stages


def gram_triplets(Ys, tau: float):
    """Singular triplets of a sparse Y with sigma > tau, plus sigma_{r+1}.

    Tier B of the oracle, for sizes where a dense Jacobi SVD per iteration is
    too slow.  The plain definition via the Gram matrix: on the smaller side,
    G = Y^T Y (or Y Y^T) = V diag(sigma^2) V^T (LAPACK's symmetric
    eigensolver, FP64), and u_i = Y v_i / sigma_i.  Singular values are
    accurate to eps * sigma_1^2 / sigma_i relative, ample for those above tau.
    Returns (U_r, sigma_r, V_r, all singular values descending).
    """
    m, n = Ys.shape
    if m >= n:
        G = (Ys.T @ Ys).toarray()
        lam, W = np.linalg.eigh(G)
        order = np.argsort(lam)[::-1]
        lam, W = lam[order], W[:, order]
        s = np.sqrt(np.maximum(lam, 0.0))
        r = int(np.count_nonzero(s > tau))
        V = W[:, :r]
        U = (Ys @ V) / s[:r] if r > 0 else np.zeros((m, 0))
    else:
        G = (Ys @ Ys.T).toarray()
        lam, W = np.linalg.eigh(G)
        order = np.argsort(lam)[::-1]
        lam, W = lam[order], W[:, order]
        s = np.sqrt(np.maximum(lam, 0.0))
        r = int(np.count_nonzero(s > tau))
        U = W[:, :r]
        V = (Ys.T @ U) / s[:r] if r > 0 else np.zeros((n, 0))
    return U, s[:r], V, s


def svt_sparse(m: int, n: int, rows, cols, vals, tau: float, delta: float,
               eps: float, maxiter: int, incr: int, kick: bool = True,
               progress=None):
    """Algorithm 1 (Section 5.1.5), tier B: sparse Y, triplets from the Gram
    matrix (``gram_triplets``); otherwise the same steps as ``svt_dense``.
    ||P_Omega M||_2 for the kick is the largest singular value from the same
    route."""
    import scipy.sparse as sp
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    norm_pm = _fro(vals)
    cap = min(m, n)
    # CSR pattern fixed; the iterate's values follow Omega's input order
    order = np.lexsort((cols, rows))
    rs, cs = rows[order], cols[order]

    def as_sparse(y):
        return sp.csr_matrix((y[order], (rs, cs)), shape=(m, n))

    sigma1 = None
    y = np.zeros(vals.shape[0])
    k0 = 0
    if kick:
        sigma1 = float(gram_triplets(as_sparse(vals), 0.0)[3][0])
        k0 = k0_kick(tau, delta, sigma1)
        y = k0 * delta * vals
    ranks, s_hist, res_hist = [], [], []
    r_prev = 0
    status = "not_converged"
    Uw = np.zeros((m, 0)); Vr = np.zeros((n, 0)); w = np.zeros(0)
    k = 0
    for k in range(1, maxiter + 1):
        U, sr, V, s = gram_triplets(as_sparse(y), tau)
        s_k = min(r_prev + 1, cap)
        while s[s_k - 1] > tau and s_k < cap:
            s_k = min(s_k + incr, cap)
        r_k = sr.shape[0]
        w = sr - tau
        Uw = U * w
        Vr = V
        e = vals - sampled_entries(Uw, Vr, rows, cols)
        res = _fro(e) / norm_pm
        ranks.append(r_k)
        s_hist.append(s_k)
        res_hist.append(res)
        if progress:
            progress(k, r_k, res)
        if res <= eps:
            status = "ok"
            break
        y = y + delta * e
        r_prev = r_k
    return dict(iters=k, k0=k0, sigma1=sigma1, ranks=ranks, s_hist=s_hist,
                residuals=res_hist, U=Uw, w=w, V=Vr, status=status, norm_pm=norm_pm)
