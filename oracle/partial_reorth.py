"""Golub-Kahan-Lanczos bidiagonalisation with partial reorthogonalisation
driven by estimates of the loss of orthogonality, in plain FP64.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may use this module.  It shares no code with the HIP
library.

Section 5.1.1 takes the triplets of Y above tau from a Lanczos
bidiagonalisation with partial reorthogonalisation (the PROPACK package).
Single-vector bidiagonalisation of Y (m x n) from a unit v_1:

    alpha_j u_j     = Y v_j   - beta_j u_{j-1}        (beta_1 u_0 = 0)
    beta_{j+1} v_{j+1} = Y^T u_j - alpha_j v_j

In exact arithmetic the u_j are orthonormal and so are the v_j; in floating
point they lose orthogonality once Ritz values converge.  Full
reorthogonalisation orthogonalises every new vector against all earlier
ones.  Partial reorthogonalisation (Simon, 1984, for the symmetric Lanczos
process; Larsen, 1998, for bidiagonalisation) does so only when an estimate
of the loss passes a level eta, and keeps the bases semi-orthogonal, which
is enough for the Ritz values and vectors to be accurate to rounding.

The estimates.  Write mu_{j,i} = u_j^T u_i and nu_{j,i} = v_j^T v_i (i < j,
mu_{j,j} = nu_{j,j} = 1).  Multiplying the first relation by u_i and using
Y^T u_i = beta_{i+1} v_{i+1} + alpha_i v_i, and the second by v_i and using
Y v_i = alpha_i u_i + beta_i u_{i-1}:

    alpha_j mu_{j,i}       = beta_{i+1} nu_{j,i+1} + alpha_i nu_{j,i} - beta_j mu_{j-1,i}
    beta_{j+1} nu_{j+1,i}  = alpha_i mu_{j,i} + beta_i mu_{j,i-1} - alpha_j nu_{j,i}

exactly for the computed vectors, up to the rounding of the step itself.
The estimate runs these recurrences on the coefficients alone and adds that
rounding as a term of size eps * c * ||Y||_est / (the divisor), with the
sign of the value it is added to (so the estimate only grows); ||Y||_est is
the largest alpha_i + beta_i seen so far, eps the unit roundoff of the
stored vectors, and c = sqrt(m + n) for vectors in FP64.  Vectors stored in
FP32 (with FP32 products, the rest in FP64, as the mixed form computes)
take c = 1: their rounding is dominated by that of their storage, which
has no systematic direction (the tests pin both choices).  A vector that is
reorthogonalised (twice against all earlier vectors of its side: classical
Gram-Schmidt applied twice) has its row of estimates set to eps.  The
policy: once the largest estimate of a new vector passes eta, that vector
and the next vector of the other side are reorthogonalised.

The rank decision is the one of ``block_krylov`` with b = 1 (Algorithm 1's,
taken strictly): stop once every Ritz value above tau and the first one at
or below it have residual bounds beta_{k+1} |p_{k,i}| of at most tol * s_1.
"""
from __future__ import annotations

import numpy as np

EPS64 = np.finfo(np.float64).eps / 2  # unit roundoff of FP64
EPS32 = 2.0 ** -24                     # unit roundoff of FP32


def _cgs2(z, Q):
    """z orthogonalised against the columns of Q by classical Gram-Schmidt,
    applied twice."""
    if Q.shape[1] == 0:
        return z
    for _ in range(2):
        z = z - Q @ (Q.T @ z)
    return z


class OmegaEstimate:
    """The estimates mu_{j, .} and nu_{j, .} of the module docstring, one row
    per vector, advanced with each new coefficient.  ``unit`` is the unit
    roundoff the new vectors are stored in, ``dim`` = m + n, ``root`` the
    factor c of the rounding term (default sqrt(dim)).  ``row_u`` /
    ``row_v`` give the row of the next vector from its norm before it is
    reorthogonalised; ``push_u`` / ``push_v`` then record its coefficient and
    its row (that row, or eps if the vector was reorthogonalised)."""

    def __init__(self, unit: float = EPS64, dim: int = 2, root=None):
        self.unit = unit
        self.root = np.sqrt(dim) if root is None else root
        self.alpha = []          # alpha[j - 1] = alpha_j
        self.beta = [0.0]        # beta[j - 1] = beta_j (beta_1 multiplies u_0 = 0)
        self.mu = []             # mu[j - 1] = estimates of u_j against u_1 .. u_{j-1}
        self.nu = [np.zeros(0)]  # nu[j - 1] = estimates of v_j against v_1 .. v_{j-1}
        self.anorm = 0.0

    def _noise(self, anorm, divisor):
        return self.unit * self.root * anorm / divisor

    def row_u(self, alpha_j: float):
        """mu_{j, 1..j-1} of u_j (j = len(alpha) + 1) from alpha_j."""
        j = len(self.alpha) + 1
        a, b = self.alpha, self.beta
        anorm = max(self.anorm, alpha_j + b[j - 1])
        nu_j = self.nu[j - 1]                       # v_j against v_1 .. v_{j-1}
        mu_prev = self.mu[j - 2] if j >= 2 else np.zeros(0)
        row = np.zeros(j - 1)
        for i in range(1, j):                       # i = 1 .. j-1
            nu_ji1 = 1.0 if i + 1 == j else nu_j[i]           # nu_{j, i+1}
            t = b[i] * nu_ji1 + a[i - 1] * nu_j[i - 1]        # beta_{i+1}, alpha_i
            mu_ji = 1.0 if i == j - 1 else mu_prev[i - 1]     # mu_{j-1, i}
            t -= b[j - 1] * mu_ji                             # beta_j
            t /= alpha_j
            row[i - 1] = t + np.copysign(self._noise(anorm, alpha_j), t)
        return row

    def push_u(self, alpha_j: float, row, reorth: bool):
        self.anorm = max(self.anorm, alpha_j + self.beta[len(self.alpha)])
        self.alpha.append(alpha_j)
        self.mu.append(np.full(row.shape, self.unit) if reorth else row)

    def row_v(self, beta_next: float):
        """nu_{j+1, 1..j} of v_{j+1} (j = len(alpha)) from beta_{j+1}."""
        j = len(self.alpha)
        a, b = self.alpha, self.beta
        anorm = max(self.anorm, a[j - 1] + beta_next)
        mu_j = self.mu[j - 1]
        nu_j = self.nu[j - 1]
        row = np.zeros(j)
        for i in range(1, j + 1):                   # i = 1 .. j
            mu_ji = 1.0 if i == j else mu_j[i - 1]            # mu_{j, i}
            t = a[i - 1] * mu_ji                              # alpha_i
            if i >= 2:
                t += b[i - 1] * mu_j[i - 2]                   # beta_i mu_{j, i-1}
            nu_ji = 1.0 if i == j else nu_j[i - 1]            # nu_{j, i}
            t -= a[j - 1] * nu_ji                             # alpha_j
            t /= beta_next
            row[i - 1] = t + np.copysign(self._noise(anorm, beta_next), t)
        return row

    def push_v(self, beta_next: float, row, reorth: bool):
        self.anorm = max(self.anorm, self.alpha[-1] + beta_next)
        self.beta.append(beta_next)
        self.nu.append(np.full(row.shape, self.unit) if reorth else row)


def gkl(Y, k: int, policy: str = "full", eta: float = 1e-10, seed: int = 0, v1=None,
        decide=None, on_step=None, store: str = "f64"):
    """k steps of the bidiagonalisation of the module docstring on Y (a
    SciPy sparse matrix or a dense array).  policy: "full" (every new vector
    orthogonalised twice against its basis), "partial" (only those the
    estimates name, see the module docstring), "none", or "given": vector h
    (h = 2(j - 1) for u_j, 2j - 1 for v_{j+1}) is orthogonalised iff
    decide(h) is true, asked before the vector is formed; on_step(j, alpha,
    beta) is called after step j with the coefficients so far (a true
    return ends the run there).  store="f32":
    products with FP32 values and vectors, vectors stored in FP32, the rest in
    FP64, and the estimate with FP32's unit roundoff and c = 1.

    Returns dict(alpha[k], beta[k + 1] (beta[0] = 0 for beta_1 u_0, beta[j]
    = beta_{j+1}), U (m x k), V (n x (k + 1)), reorth_u, reorth_v (bool per
    vector: u_j, v_{j+1}), est_u[j] / est_v[j] (the largest estimate of u_j
    / v_{j+1} before any reorthogonalisation of it), loss_u[j] / loss_v[j]
    (the largest |u_j^T u_i| / |v_{j+1}^T v_i| actually left)."""
    m, n = Y.shape
    f32 = store == "f32"
    vt = np.float32 if f32 else np.float64
    Ys = Y.astype(np.float32) if f32 else Y
    Yt = Ys.T

    def prod(A, x):
        return np.asarray(A @ x, dtype=np.float64)

    def f64(B):
        return np.asarray(B, dtype=np.float64)

    if v1 is None:
        v1 = np.random.default_rng(seed).standard_normal(n)
    U = np.zeros((m, k), vt)
    V = np.zeros((n, k + 1), vt)
    V[:, 0] = v1 / np.linalg.norm(v1)
    alpha = np.zeros(k)
    beta = np.zeros(k + 1)
    est = OmegaEstimate(EPS32, m + n, 1.0) if f32 else OmegaEstimate(EPS64, m + n)
    out = dict(reorth_u=[], reorth_v=[], est_u=[], est_v=[], loss_u=[], loss_v=[])
    force_u = force_v = False
    for j in range(k):
        # alpha_{j+1} u_{j+1} = Y v_{j+1} - beta_{j+1} u_j
        z = prod(Ys, V[:, j])
        if j > 0:
            z = z - beta[j] * U[:, j - 1]
        row = est.row_u(np.linalg.norm(z))
        e_u = float(np.max(np.abs(row))) if row.size else 0.0
        if policy == "given":
            do = bool(decide(2 * j)) and j > 0
        else:
            do = j > 0 and (policy == "full" or (policy == "partial" and (e_u > eta or force_u)))
        force_u = False
        if do:
            z = _cgs2(z, f64(U[:, :j]))
            force_v = policy == "partial" and e_u > eta
        alpha[j] = np.linalg.norm(z)
        U[:, j] = z / alpha[j]
        est.push_u(alpha[j], row, do)
        out["reorth_u"].append(do)
        out["est_u"].append(e_u)
        out["loss_u"].append(float(np.max(np.abs(f64(U[:, :j]).T @ U[:, j]))) if j else 0.0)
        # beta_{j+2} v_{j+2} = Y^T u_{j+1} - alpha_{j+1} v_{j+1}
        z = prod(Yt, U[:, j]) - alpha[j] * V[:, j]
        row = est.row_v(np.linalg.norm(z))
        e_v = float(np.max(np.abs(row)))
        if policy == "given":
            do = bool(decide(2 * j + 1))
        else:
            do = policy == "full" or (policy == "partial" and (e_v > eta or force_v))
        force_v = False
        if do:
            z = _cgs2(z, f64(V[:, :j + 1]))
            force_u = policy == "partial" and e_v > eta
        beta[j + 1] = np.linalg.norm(z)
        V[:, j + 1] = z / beta[j + 1]
        est.push_v(beta[j + 1], row, do)
        out["reorth_v"].append(do)
        out["est_v"].append(e_v)
        out["loss_v"].append(float(np.max(np.abs(f64(V[:, :j + 1]).T @ V[:, j + 1]))))
        if on_step is not None and on_step(j + 1, alpha[:j + 1], beta[:j + 2]):
            k = j + 1                                 # the caller stops here
            break
    out.update(alpha=alpha[:k], beta=beta[:k + 1], U=U[:, :k], V=V[:, :k + 1])
    for key in ("reorth_u", "reorth_v"):
        out[key] = np.array(out[key], dtype=bool)
    for key in ("est_u", "est_v", "loss_u", "loss_v"):
        out[key] = np.array(out[key])
    return out


def ritz(alpha, beta, k: int):
    """Singular values, residual bounds and singular vectors of B_k = U_k^T Y
    V_k (upper bidiagonal: alpha_1 .. alpha_k on the diagonal, beta_2 ..
    beta_k above it, from Y v_j = alpha_j u_j + beta_j u_{j-1}).  With B_k = P
    diag(s) Q^T, Y V_k q_i = s_i U_k p_i and |Y^T U_k p_i - s_i V_k q_i| =
    beta_{k+1} |p_i[k]|, the residual bound returned."""
    B = np.zeros((k, k))
    B[np.arange(k), np.arange(k)] = alpha[:k]
    for i in range(1, k):
        B[i - 1, i] = beta[i]        # Y v_{i+1} = beta_{i+1} u_i + alpha_{i+1} u_{i+1}
    P, s, Qt = np.linalg.svd(B)
    resid = abs(beta[k]) * np.abs(P[k - 1, :])
    return s, resid, P, Qt.T


def decide(Y, tau: float, tol: float = 1e-12, kmax: int = 1000, policy: str = "full",
           eta: float = 1e-10, seed: int = 0):
    """Run the bidiagonalisation on Y until Algorithm 1's rank decision
    (strict, as ``block_krylov.block_gkl`` with b = 1) is certain.  Returns
    dict(steps, rank, sigma (Ritz values through the first at or below tau),
    resid, reorth (the number of vectors reorthogonalised), vectors (2
    steps), U, V (the Ritz vectors of the values above tau), run) or None."""
    m, n = Y.shape
    kmax = min(kmax, m, n)
    found = {}

    def check(k, alpha, beta):
        s, res, P, Q = ritz(alpha, beta, k)
        r = int(np.count_nonzero(s > tau))
        if k == min(m, n) or (r < k and np.all(res[:r + 1] <= tol * s[0])):
            found.update(k=k, s=s, res=res, P=P, Q=Q, r=r)
            return True
        return False

    run = gkl(Y, kmax, policy=policy, eta=eta, seed=seed, on_step=check)
    if not found:
        return None
    k, r, P, Q = found["k"], found["r"], found["P"], found["Q"]
    nre = int(run["reorth_u"][:k].sum() + run["reorth_v"][:k].sum())
    return dict(steps=k, rank=r, sigma=found["s"][:r + 1], resid=found["res"][:r + 1], reorth=nre,
                vectors=2 * k, U=np.asarray(run["U"][:, :k], dtype=np.float64) @ P[:, :r],
                V=np.asarray(run["V"][:, :k], dtype=np.float64) @ Q[:, :r], run=run)
