"""Block Golub-Kahan-Lanczos bidiagonalisation (b vectors per step) with full
reorthogonalisation, in plain FP64: an experiment on how many sparse
products a block method needs to make Algorithm 1's rank decision.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may use this module.  It shares no code with the HIP
library.

Section 5.1.1 computes the triplets of Y above tau by single-vector
bidiagonalisation.  The block form (Golub, Luk and Overton, 1981) starts
from b orthonormal columns V_1 and, for j = 1, 2, ...,

    U_j R_j     = Y V_j - U_{j-1} S_j^T          (QR of the right-hand side)
    V_{j+1} S_{j+1} = Y^T U_j - V_j R_j^T        (QR again)

with every new block orthogonalised twice against all earlier blocks of its
side before the QR.  Then Y V_k = U_k T_k with T_k (kb x kb) block upper
bidiagonal: R_j on the diagonal, S_{j+1}^T above it.  For T_k = P diag(s) Q^T
the pair (U_k p_i, V_k q_i) has Y V_k q_i = s_i U_k p_i exactly and
|Y^T U_k p_i - s_i V_k q_i| = |S_{k+1} p_i[last block]|, the residual bound
used below.  The decision is Algorithm 1's, taken strictly: stop once every
Ritz value above tau and the first one below it have a residual bound of at
most tol * s_1 (the single-vector case b = 1 is the rule the GPU solver
applies with decide_margin >= 1).  Each step costs 2b sparse products.
"""
from __future__ import annotations

import numpy as np


def _orth_against(Z, blocks):
    for _ in range(2):
        for Q in blocks:
            Z = Z - Q @ (Q.T @ Z)
    return Z


def block_gkl(Y, b: int, tau: float, tol: float = 1e-12, kmax: int = 1000, seed: int = 0):
    """The block bidiagonalisation above on the sparse Y (scipy CSR, m x n).
    Returns dict(steps, products (= 2 b steps), rank, sigma (the Ritz values
    up to the first one below tau), resid (their residual bounds)), or None
    if the decision is not reached within kmax steps."""
    m, n = Y.shape
    Yt = Y.T.tocsr()
    rng = np.random.default_rng(seed)
    V = [np.linalg.qr(rng.standard_normal((n, b)))[0]]
    U, R, S = [], [], []
    for j in range(kmax):
        Z = Y @ V[j]
        if j > 0:
            Z = Z - U[j - 1] @ S[j - 1].T
        Uj, Rj = np.linalg.qr(_orth_against(Z, U))
        U.append(Uj)
        R.append(Rj)
        W = Yt @ Uj - V[j] @ Rj.T
        Vn, Sn = np.linalg.qr(_orth_against(W, V))
        V.append(Vn)
        S.append(Sn)
        k = j + 1
        K = k * b
        T = np.zeros((K, K))
        for i in range(k):
            T[i * b:(i + 1) * b, i * b:(i + 1) * b] = R[i]
            if i + 1 < k:
                T[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = S[i].T
        P, s, _ = np.linalg.svd(T)
        resid = np.linalg.norm(S[k - 1] @ P[(k - 1) * b:k * b, :], axis=0)
        r = int(np.count_nonzero(s > tau))
        if r < K and np.all(resid[:r + 1] <= tol * s[0]):
            return dict(steps=k, products=2 * b * k, rank=r, sigma=s[:r + 1].copy(),
                        resid=resid[:r + 1].copy())
        if min(m, n) <= K + b:
            break
    return None
