"""Write the oracle's results for the seeded square workloads.

Calls only the CPU oracle on the seeded workloads; the HIP path's tests
compare against the stored files.  Run from the repository root:

    python tests/golden/make_oracle_goldens.py 1      # 400 x 400, rank 10: tier A (dense Jacobi)
    python tests/golden/make_oracle_goldens.py 2      # 5000 x 5000, rank 10: tier B (Gram matrix)
    python tests/golden/make_oracle_goldens.py 2 60   # the same, X at iteration 60 (eps = 0)
    python tests/golden/make_oracle_goldens.py 3 40   # 10000 x 10000, rank 50: tier B, X at iteration 40
    python tests/golden/make_oracle_goldens.py 3 C    # the same, complete run: tier C (library partial SVD)
    python tests/golden/make_oracle_goldens.py 4 C    # 30000 x 30000, rank 10: tier C, complete run,
                                                      # plus X at iterations 20 and 60
    python tests/golden/make_oracle_goldens.py dantzig  # Figure 3's workload, the Dantzig selector
    python tests/golden/make_oracle_goldens.py serving  # four serving-stream requests, X at iteration 30

With a second argument k the run stops after k iterations with eps = 0, and
the file holds X^k: a fixed-iteration comparison point for trajectories
that amplify rounding differences (near the end of the 5000 x 5000 run the
rank of X flips between 10, 11 and 12, and two solvers that differ only in
rounding part ways).  With "C" the complete run of tier C is stored, and for
the 30000 x 30000 workload also its X^20 and X^60 (the loop is the same up to
there whatever eps is, so these equal runs stopped at 20 and 60 with
eps = 0).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workload  # noqa: E402
from oracle.krylov import svt_krylov  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

SNAPSHOTS = {4: (20, 60)}
# tier C's X^k checked against a stored tier-B X^k of the same workload (the
# comparison is stored; the factors are not stored twice)
CROSS_CHECK = {3: 40}


def _save(path, U, w, V, iters, k0, sigma1, ranks, s_hist, residuals, seconds, tier, **extra):
    np.savez_compressed(path, U=U, w=w, V=V, iters=iters, k0=k0, sigma1=sigma1,
                        ranks=np.array(ranks), s_hist=np.array(s_hist),
                        residuals=np.array(residuals), seconds=seconds, tier=tier, **extra)
    print(f"wrote {path}: tier {tier}, {iters} iterations, k0 {k0}", flush=True)


# the Dantzig-selector run of Figure 3's workload: half the paper's step
# (with delta = 1.2 / p the two-multiplier iteration oscillates there) and
# the eq. (5.10) consistency stop
DANTZIG_STEP_SCALE = 0.5


def dantzig():
    from oracle.dantzig import svt_dantzig
    p = workload.dantzig_fig3(seed=0)
    t = time.time()
    out = svt_dantzig(p.m, p.n, p.rows, p.cols, p.vals, p.noise_sigma, p.tau, DANTZIG_STEP_SCALE * p.delta,
                      p.eps, p.maxiter, p.incr, partial="sparse", stop="noisy", noise_sigma=p.noise_sigma,
                      progress=lambda k, r, res: print(f"  iteration {k}: rank {r}, violation {res:.3e}",
                                                       flush=True))
    _save(os.path.join(HERE, "oracle_dantzig_fig3.npz"), out["U"], out["w"], out["V"], out["iters"], out["k0"],
          out["sigma1"], out["ranks"], out["s_hist"], out["residuals"], time.time() - t, "C",
          delta=DANTZIG_STEP_SCALE * p.delta, E=p.noise_sigma, status=out["status"])


# requests of the serving stream (workload.serving_trace, seed 0) compared at
# a fixed iteration: square-ish, wide and tall members inside the method's regime
SERVING_REQUESTS = (5, 8, 15, 17)
SERVING_K = 30


def serving():
    trace = workload.serving_trace(32, seed=0, rate=1.0)
    out = {}
    for i in SERVING_REQUESTS:
        sp_ = trace[i][1]
        p = workload.gaussian_lowrank(sp_["m"], sp_["n"], sp_["r"], sp_["nnz"], sp_["seed"],
                                      noise_sigma=sp_["noise_sigma"], maxiter=500)
        t = time.time()
        o = svt_krylov(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, 0.0, SERVING_K, p.incr)
        print(f"request {i}: {p.m} x {p.n}, r {p.r}, |Omega| {p.nnz}: {time.time() - t:.0f} s, ranks {o['ranks'][-3:]}",
              flush=True)
        for key in ("U", "w", "V"):
            out[f"r{i}_{key}"] = o[key]
        out[f"r{i}_ranks"] = np.array(o["ranks"])
        out[f"r{i}_residuals"] = np.array(o["residuals"])
        out[f"r{i}_k0"] = o["k0"]
    np.savez_compressed(os.path.join(HERE, f"oracle_serving_k{SERVING_K}.npz"), requests=np.array(SERVING_REQUESTS),
                        k=SERVING_K, tier="C", **out)


def main(cfg: int, arg: str = "0"):
    p = workload.config(cfg, seed=0)
    t = time.time()

    def progress(k, r, res, *rest):
        print(f"  iteration {k}: rank {r}, residual {res:.3e}, {time.time() - t:.0f} s", flush=True)

    if arg == "C":
        snaps = tuple(SNAPSHOTS.get(cfg, ())) + ((CROSS_CHECK[cfg],) if cfg in CROSS_CHECK else ())
        out = svt_krylov(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr,
                         progress=progress, keep_iterates_at=snaps)
        dt = time.time() - t
        extra = {}
        if cfg in CROSS_CHECK and CROSS_CHECK[cfg] in out["snapshots"]:
            from tests.helpers import rel_diff_factored
            kk = CROSS_CHECK[cfg]
            b = np.load(os.path.join(HERE, f"oracle_config{cfg}_k{kk}.npz"))
            U, w, V = out["snapshots"][kk]
            extra = dict(cross_k=kk, cross_tier=str(b["tier"]),
                         cross_x_rel_diff=rel_diff_factored(U, V, b["U"], b["V"]),
                         cross_ranks_equal=bool(list(b["ranks"]) == out["ranks"][:kk]),
                         cross_s_equal=bool(list(b["s_hist"]) == out["s_hist"][:kk]),
                         cross_res_rel_diff=float(np.max(np.abs(np.array(out["residuals"][:kk]) - b["residuals"])
                                                         / b["residuals"])))
            print(f"cross-check at k = {kk} against tier {extra['cross_tier']}: {extra}", flush=True)
        for kk in SNAPSHOTS.get(cfg, ()):
            if kk in out["snapshots"]:
                U, w, V = out["snapshots"][kk]
                _save(os.path.join(HERE, f"oracle_config{cfg}_k{kk}.npz"), U, w, V, kk, out["k0"],
                      out["sigma1"], out["ranks"][:kk], out["s_hist"][:kk], out["residuals"][:kk],
                      float(np.sum(out["seconds"][:kk])), "C")
        _save(os.path.join(HERE, f"oracle_config{cfg}.npz"), out["U"], out["w"], out["V"], out["iters"],
              out["k0"], out["sigma1"], out["ranks"], out["s_hist"], out["residuals"], dt, "C", **extra)
        return
    kfix = int(arg)
    eps, maxiter = (0.0, kfix) if kfix > 0 else (p.eps, p.maxiter)
    if cfg == 1:
        out = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, eps,
                               maxiter, p.incr)
        tier = "A"
    else:
        out = oracle.svt_sparse(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, eps,
                                maxiter, p.incr, progress=progress)
        tier = "B"
    dt = time.time() - t
    suffix = f"_k{kfix}" if kfix > 0 else ""
    _save(os.path.join(HERE, f"oracle_config{cfg}{suffix}.npz"), out["U"], out["w"], out["V"], out["iters"],
          out["k0"], out["sigma1"], out["ranks"], out["s_hist"], out["residuals"], dt, tier)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "dantzig":
        dantzig()
    elif len(sys.argv) > 1 and sys.argv[1] == "serving":
        serving()
    else:
        main(int(sys.argv[1]) if len(sys.argv) > 1 else 1, sys.argv[2] if len(sys.argv) > 2 else "0")
