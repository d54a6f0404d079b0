"""Seeded synthetic matrix-completion workloads.

This module only draws inputs: it holds none of the completion method's
arithmetic, and both the HIP path and the CPU oracle take their inputs from it.

Data model (Section 5.2.1, "Linear equality constraints"): an n1 x n2 matrix
of rank r is the product M = M_L M_R^T of two factors with i.i.d. standard
Gaussian entries, and the observed set Omega is drawn uniformly at random among
all index sets of its cardinality (sampling without replacement).  The number
of samples is a multiple c of the degrees of freedom d_r = r(n1 + n2 - r)
(Section 1.1 for the square case, d_r = r(2n - r)).

The default parameters follow Section 5.2.1: tau = 5n (tau = 5 sqrt(n1 n2) for
rectangular matrices), delta = 1.2 n1 n2 / |Omega| (eq. "heuristic" of
Section 5.1.2), eps = 1e-4 (eq. "stop"), ell = 5 (Section 5.1.1).

Draw order for one problem, from ``numpy.random.default_rng(seed)``:
M_L, then M_R, then Omega, then (optional) noise.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem",
    "degrees_of_freedom",
    "sample_omega",
    "gaussian_lowrank",
    "config",
    "CONFIGS",
    "serving_trace",
    "TABLE1_RANK_OVERSAMPLING",
    "full_observation",
    "dense_random_iterate",
    "dantzig_fig3",
    "SensingProblem",
    "sparse_sensing",
]


@dataclasses.dataclass
class Problem:
    """One completion problem: dimensions, Omega in COO form and P_Omega(M)."""

    m: int
    n: int
    r: int
    rows: np.ndarray      # int32[nnz], row index of each observed entry
    cols: np.ndarray      # int32[nnz], column index of each observed entry
    vals: np.ndarray      # float64[nnz], observed values M_ij (plus noise if any)
    ML: np.ndarray        # float64[m, r] left factor of the truth
    MR: np.ndarray        # float64[n, r] right factor of the truth
    tau: float
    delta: float
    eps: float
    maxiter: int
    incr: int
    name: str = ""
    noise_sigma: float = 0.0

    @property
    def nnz(self) -> int:
        return int(self.rows.shape[0])


def degrees_of_freedom(m: int, n: int, r: int) -> int:
    """d_r = r (m + n - r): parameters of an m x n rank-r matrix (Section 1.1)."""
    return r * (m + n - r)


def sample_omega(rng: np.random.Generator, m: int, n: int, nnz: int) -> np.ndarray:
    """nnz distinct linear indices in [0, m*n), uniform without replacement.

    Drawn by rejection: draw uniform int64 indices, drop repeats, draw again for
    the shortfall.  The result is sorted (row-major order).
    """
    total = m * n
    if nnz > total:
        raise ValueError("nnz exceeds m*n")
    if nnz * 2 > total:
        # dense case: a permutation prefix is cheaper than rejection
        return np.sort(rng.permutation(total)[:nnz]).astype(np.int64)
    picked = np.unique(rng.integers(0, total, size=nnz, dtype=np.int64))
    while picked.shape[0] < nnz:
        extra = rng.integers(0, total, size=nnz - picked.shape[0], dtype=np.int64)
        picked = np.unique(np.concatenate([picked, extra]))
    if picked.shape[0] > nnz:
        # unique() sorted the candidates; keep a uniformly random subset
        keep = np.sort(rng.permutation(picked.shape[0])[:nnz])
        picked = picked[keep]
    return picked


def _observed_values(ML: np.ndarray, MR: np.ndarray, rows: np.ndarray,
                     cols: np.ndarray, chunk: int = 1 << 20) -> np.ndarray:
    """Entries M_ij = <M_L[i], M_R[j]> of the truth at the observed positions."""
    out = np.empty(rows.shape[0], dtype=np.float64)
    for s in range(0, rows.shape[0], chunk):
        e = min(s + chunk, rows.shape[0])
        out[s:e] = np.einsum("ij,ij->i", ML[rows[s:e]], MR[cols[s:e]])
    return out


def gaussian_lowrank(m: int, n: int, r: int, nnz: int, seed: int = 0, *,
                     tau: float | None = None, delta: float | None = None,
                     eps: float = 1e-4, maxiter: int = 500, incr: int = 5,
                     noise_sigma: float = 0.0, shuffle: bool = False,
                     name: str = "") -> Problem:
    """Gaussian rank-r truth observed on a uniform random Omega.

    ``shuffle`` returns the COO triplets in a random order instead of
    row-major order (the library must not depend on the order).
    """
    rng = np.random.default_rng(seed)
    ML = rng.standard_normal((m, r))
    MR = rng.standard_normal((n, r))
    lin = sample_omega(rng, m, n, nnz)
    rows = (lin // n).astype(np.int32)
    cols = (lin % n).astype(np.int32)
    vals = _observed_values(ML, MR, rows, cols)
    if noise_sigma > 0.0:
        vals = vals + noise_sigma * rng.standard_normal(nnz)
    if shuffle:
        order = rng.permutation(nnz)
        rows, cols, vals = rows[order], cols[order], vals[order]
    if tau is None:
        tau = 5.0 * math.sqrt(float(m) * float(n))
    if delta is None:
        delta = 1.2 * float(m) * float(n) / float(nnz)
    return Problem(m=m, n=n, r=r, rows=rows, cols=cols, vals=vals, ML=ML, MR=MR,
                   tau=float(tau), delta=float(delta), eps=float(eps),
                   maxiter=int(maxiter), incr=int(incr), name=name,
                   noise_sigma=float(noise_sigma))


# The four single-solve workloads: (n, r, |Omega| / d_r).  Sizes follow the
# shapes of Table 1; the 30000 x 30000, rank-10, 6 d_r case is Table 1's last row.
CONFIGS = {
    1: dict(n=400, r=10, c=6, name="svt-400sq-r10-6dr"),
    2: dict(n=5000, r=10, c=5, name="svt-5000sq-r10-5dr"),
    3: dict(n=10000, r=50, c=4, name="svt-10000sq-r50-4dr"),
    4: dict(n=30000, r=10, c=6, name="svt-30000sq-r10-6dr"),
}


# Table 2 (Section 5.2.1): n = 1000 with (r, |Omega| / d_r) = (10, 6),
# (50, 4), (100, 3), at noise ratios 1e-2, 1e-1 and 1.
TABLE2_RANK_OVERSAMPLING = ((10, 6.0), (50, 4.0), (100, 3.0))
TABLE2_NOISE_RATIOS = (1e-2, 1e-1, 1.0)


def noisy_lowrank(n: int, r: int, c: float, noise_ratio: float, seed: int = 0, *,
                  eps: float = 1e-4, maxiter: int = 500) -> Problem:
    """Gaussian rank-r n x n truth on a uniform random Omega of c d_r entries,
    observed as B = M + Z with Z white Gaussian noise of standard deviation
    sigma = noise_ratio |P_Omega M|_F / sqrt(|Omega|), so that the noise ratio
    |P_Omega Z|_F / |P_Omega M|_F is noise_ratio in expectation (Section
    5.2.1's model).  ``vals`` holds B; ``clean`` (an extra attribute) holds
    P_Omega M, and ``noise_sigma`` the sigma to give the stop rule."""
    nnz = int(round(c * degrees_of_freedom(n, n, r)))
    rng = np.random.default_rng(seed)
    ML = rng.standard_normal((n, r))
    MR = rng.standard_normal((n, r))
    lin = sample_omega(rng, n, n, nnz)
    rows = (lin // n).astype(np.int32)
    cols = (lin % n).astype(np.int32)
    clean = _observed_values(ML, MR, rows, cols)
    sigma = noise_ratio * float(np.linalg.norm(clean)) / math.sqrt(float(nnz))
    vals = clean + sigma * rng.standard_normal(nnz)
    p = Problem(m=n, n=n, r=r, rows=rows, cols=cols, vals=vals, ML=ML, MR=MR,
                tau=5.0 * float(n), delta=1.2 * float(n) * float(n) / float(nnz), eps=float(eps),
                maxiter=int(maxiter), incr=5, name=f"svt-noisy-{n}sq-r{r}-nr{noise_ratio:g}",
                noise_sigma=float(sigma))
    p.clean = clean
    return p


def dantzig_fig3(n: int = 1000, r: int = 10, c: float = 5.0, seed: int = 0, *,
                 eps: float = 1e-4, maxiter: int = 500) -> Problem:
    """The linear-inequality experiment of Section 5.2.2 (Figure 3): a
    Gaussian rank-r n x n truth on a uniform random Omega of c d_r entries,
    observed as B = M + Z with white Gaussian Z of standard deviation
    sigma = 0.1 sum_{Omega} |M_ij| / |Omega| (one tenth of a typical observed
    entry), tau = 5n, delta = 1.2 n^2 / |Omega|.  ``vals`` holds B,
    ``clean`` holds P_Omega M, ``noise_sigma`` holds sigma (the tolerance E
    of every constraint |X_ij - B_ij| <= E).  Draw order: M_L, M_R, Omega,
    noise."""
    nnz = int(round(c * degrees_of_freedom(n, n, r)))
    rng = np.random.default_rng(seed)
    ML = rng.standard_normal((n, r))
    MR = rng.standard_normal((n, r))
    lin = sample_omega(rng, n, n, nnz)
    rows = (lin // n).astype(np.int32)
    cols = (lin % n).astype(np.int32)
    clean = _observed_values(ML, MR, rows, cols)
    sigma = 0.1 * float(np.mean(np.abs(clean)))
    vals = clean + sigma * rng.standard_normal(nnz)
    p = Problem(m=n, n=n, r=r, rows=rows, cols=cols, vals=vals, ML=ML, MR=MR,
                tau=5.0 * float(n), delta=1.2 * float(n) * float(n) / float(nnz), eps=float(eps),
                maxiter=int(maxiter), incr=5, name=f"svt-dantzig-{n}sq-r{r}-{c:g}dr",
                noise_sigma=float(sigma))
    p.clean = clean
    return p


@dataclasses.dataclass
class SensingProblem:
    """Linear measurements b = A(M) of a rank-r matrix (Section 3.1): entry
    positions of the support S (srows, scols, row-major, distinct) and the
    p x |S| measurement matrix G in CSR form (gptr, gidx into S, gval), so
    that b_i = sum_s G[i, s] M[srows[s], scols[s]]."""

    m: int
    n: int
    r: int
    srows: np.ndarray
    scols: np.ndarray
    gptr: np.ndarray
    gidx: np.ndarray
    gval: np.ndarray
    b: np.ndarray
    ML: np.ndarray
    MR: np.ndarray
    tau: float
    delta: float
    eps: float
    maxiter: int
    incr: int
    name: str = ""

    @property
    def p(self) -> int:
        return int(self.b.shape[0])

    def G(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.gval, self.gidx, self.gptr), shape=(self.p, self.srows.shape[0]))


def sparse_sensing(m: int, n: int, r: int, p: int, c: int = 4, seed: int = 0, *,
                   eps: float = 1e-4, maxiter: int = 500) -> SensingProblem:
    """A Gaussian rank-r m x n truth seen through p measurements, each a
    random combination of c distinct entries at uniform positions with
    N(0, 1/c) weights (so E[A* A] = p / (m n) I, as E[P_Omega] = |Omega| /
    (m n) I for sampling).  tau = 5 sqrt(m n) and delta = 1.2 m n / p carry
    the completion choices over (Section 5.2.1).  Draw order: M_L, M_R, the
    positions, the weights."""
    rng = np.random.default_rng(seed)
    ML = rng.standard_normal((m, r))
    MR = rng.standard_normal((n, r))
    pos = np.empty((p, c), dtype=np.int64)
    for i in range(p):
        pos[i] = rng.choice(m * n, size=c, replace=False)
    wts = rng.standard_normal((p, c)) / math.sqrt(c)
    support, inv = np.unique(pos.ravel(), return_inverse=True)
    srows = (support // n).astype(np.int32)
    scols = (support % n).astype(np.int32)
    gidx = inv.reshape(p, c).astype(np.int32)
    order = np.argsort(gidx, axis=1)
    gidx = np.take_along_axis(gidx, order, axis=1)
    gval = np.take_along_axis(wts, order, axis=1)
    gptr = np.arange(0, p * c + 1, c, dtype=np.int64)
    ms = _observed_values(ML, MR, srows, scols)
    b = (gval * ms[gidx]).sum(axis=1)
    return SensingProblem(m=m, n=n, r=r, srows=srows, scols=scols, gptr=gptr, gidx=gidx.ravel(),
                          gval=gval.ravel(), b=b, ML=ML, MR=MR, tau=5.0 * math.sqrt(float(m) * float(n)),
                          delta=1.2 * float(m) * float(n) / float(p), eps=float(eps), maxiter=int(maxiter),
                          incr=5, name=f"sensing-{m}x{n}-r{r}-p{p}-c{c}")


def config(idx: int, seed: int = 0) -> Problem:
    """Square workload ``idx`` (1..4): tau = 5n, delta = 1.2 n^2/|Omega|."""
    c = CONFIGS[idx]
    n, r = c["n"], c["r"]
    nnz = c["c"] * degrees_of_freedom(n, n, r)
    return gaussian_lowrank(n, n, r, nnz, seed, tau=5.0 * n, eps=1e-4,
                            maxiter=500, incr=5, name=c["name"])


def full_observation(m: int, n: int, sigma: np.ndarray, seed: int = 0):
    """A matrix with prescribed singular values, observed everywhere.

    Returns (Problem, U, sigma, V) with M = U diag(sigma) V^T; U and V have
    orthonormal columns (QR of Gaussian matrices).  With Omega = every entry,
    P_Omega is the identity and delta = 1.2 n1 n2 / m equals 1.2.
    """
    rng = np.random.default_rng(seed)
    k = sigma.shape[0]
    U, _ = np.linalg.qr(rng.standard_normal((m, k)))
    V, _ = np.linalg.qr(rng.standard_normal((n, k)))
    lin = np.arange(m * n, dtype=np.int64)
    rows = (lin // n).astype(np.int32)
    cols = (lin % n).astype(np.int32)
    Mfull = (U * sigma) @ V.T
    vals = Mfull[rows, cols].copy()
    tau = 5.0 * math.sqrt(float(m) * float(n))
    prob = Problem(m=m, n=n, r=k, rows=rows, cols=cols, vals=vals, ML=U * sigma,
                   MR=V, tau=tau, delta=1.2, eps=1e-4, maxiter=500, incr=5,
                   name=f"fullobs-{m}x{n}")
    return prob, U, sigma, V


def dense_random_iterate(prob: Problem, seed: int = 1) -> np.ndarray:
    """Seeded Gaussian values on Omega: a generic sparse iterate for kernel tests."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(prob.nnz)


# (rank, |Omega| / d_r) pairs of the paper's Table 1 at n >= 5000
TABLE1_RANK_OVERSAMPLING = ((10, 6.0), (50, 5.0), (100, 4.0))


def serving_trace(count: int, seed: int = 0, *, mn_range=(500, 8000),
                  ranks=(5, 10, 20, 50), c_range=(3.0, 6.0), pairs=None,
                  rate: float = 1.0, noise_frac: float = 0.0, noise_sigma: float = 0.01,
                  max_fill: float = 0.6, max_aspect=None):
    """Poisson stream of mixed completion requests.

    Each request draws m, n uniform integers in ``mn_range``; r from
    ``ranks`` and c uniform in ``c_range`` (or, with ``pairs`` given, a
    (r, c) pair from it, e.g. TABLE1_RANK_OVERSAMPLING); and |Omega| =
    floor(c r (m + n - r)).  A request whose |Omega| would exceed
    ``max_fill`` * m n, or whose aspect ratio max(m, n) / min(m, n) exceeds
    ``max_aspect`` (when given), is drawn again.  tau = 5 sqrt(m n), delta =
    1.2 m n / |Omega|, eps = 1e-4.  Arrival gaps are exponential with mean
    1/rate seconds.  Returns a list of (arrival_time_s, spec) where spec is a
    dict of problem parameters and a per-request seed;
    ``gaussian_lowrank(**spec)`` materialises it.

    With the default ranges some requests fall outside the regime of Table 1
    (c near 3 at a sampling density of a few percent, or c near 5 at rank 5
    or 10): with delta = 1.2 / p Algorithm 1 then oscillates or stalls on
    them, which a server has to bound.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        while True:
            m = int(rng.integers(mn_range[0], mn_range[1] + 1))
            n = int(rng.integers(mn_range[0], mn_range[1] + 1))
            if pairs is None:
                r = int(ranks[int(rng.integers(0, len(ranks)))])
                c = float(rng.uniform(c_range[0], c_range[1]))
            else:
                r, c = pairs[int(rng.integers(0, len(pairs)))]
            nnz = int(math.floor(c * degrees_of_freedom(m, n, r)))
            if nnz > max_fill * m * n:
                continue
            if max_aspect is not None and max(m, n) > max_aspect * min(m, n):
                continue
            break
        noisy = bool(rng.uniform() < noise_frac)
        t += float(rng.exponential(1.0 / rate)) if rate > 0 else 0.0
        spec = dict(m=m, n=n, r=int(r), nnz=nnz, seed=int(seed * 1000003 + i),
                    noise_sigma=noise_sigma if noisy else 0.0,
                    name=f"req{i}")
        out.append((t, spec))
    return out
