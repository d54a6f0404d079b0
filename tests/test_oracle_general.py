"""The oracle's general-operator iteration (Section 3.1, eq. (3.3)) pinned by
what the paper and the mathematics fix:

* A = the sampling operator (G = identity on S = Omega): the iteration is
  Algorithm 1's (Section 3.1 shows the two coincide with Y^k = A*(y^k)), so
  it reproduces the completion oracle exactly;
* Theorem 4.4 (F affine, L(F) = ||A||_2 = ||G||_2, 0 < delta < 2 / ||A||^2):
  the limit satisfies the KKT conditions of problem (3.1) -- A(X) = b and
  X = D_tau(A*(y)) checked with LAPACK's SVD -- which make it the unique
  solution (the objective is strongly convex);
* the kick: the run from y = 0 equals the kicked run shifted by k0.
"""
import numpy as np
import scipy.sparse as sp

import oracle
import workload
from oracle.general import adjoint, svt_general
from tests.helpers import rel_diff_factored


def test_sampling_operator_is_algorithm_1():
    p = workload.gaussian_lowrank(60, 45, 3, 1500, 2, maxiter=300)
    G = sp.identity(p.nnz, format="csr")
    g = svt_general(p.m, p.n, p.rows, p.cols, G, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr)
    a = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr)
    assert (g["iters"], g["k0"], g["status"]) == (a["iters"], a["k0"], a["status"])
    assert g["ranks"] == a["ranks"] and g["s_hist"] == a["s_hist"]
    np.testing.assert_allclose(g["residuals"], a["residuals"], rtol=1e-12)
    assert rel_diff_factored(g["U"], g["V"], a["U"], a["V"]) <= 1e-12


def test_kkt_conditions_at_the_limit():
    q = workload.sparse_sensing(30, 24, 2, 5 * 2 * (30 + 24 - 2), 3, seed=5)
    G = q.G()
    normA2 = np.linalg.norm(G.toarray(), 2) ** 2
    tau = 20.0
    out = svt_general(q.m, q.n, q.srows, q.scols, G, q.b, tau, 1.9 / normA2, 1e-13, 40000, q.incr)
    assert out["status"] == "ok"
    X = out["U"] @ out["V"].T
    # feasibility A(X) = b
    assert np.linalg.norm(G @ X[q.srows, q.scols] - q.b) <= 1e-12 * np.linalg.norm(q.b)
    # stationarity: X = D_tau(A*(y)), the shrinkage with LAPACK
    Uf, s, Vt = np.linalg.svd(adjoint(q.m, q.n, q.srows, q.scols, G, out["y"]), full_matrices=False)
    Xref = (Uf * np.maximum(s - tau, 0.0)) @ Vt
    assert np.linalg.norm(X - Xref) <= 1e-8 * np.linalg.norm(Xref)


def test_kick_equals_unskipped_run_shifted():
    q = workload.sparse_sensing(40, 30, 2, 5 * 2 * 68, 3, seed=3)
    G = q.G()
    a = svt_general(q.m, q.n, q.srows, q.scols, G, q.b, q.tau, q.delta, q.eps, 150, q.incr)
    k0 = a["k0"]
    b = svt_general(q.m, q.n, q.srows, q.scols, G, q.b, q.tau, q.delta, q.eps, 150 + k0, q.incr, kick=False)
    assert k0 >= 1 and b["ranks"][:k0] == [0] * k0
    assert b["ranks"][k0:] == a["ranks"]
    np.testing.assert_allclose(b["residuals"][k0:], a["residuals"], rtol=1e-9)
    assert rel_diff_factored(b["U"], b["V"], a["U"], a["V"]) <= 1e-9
