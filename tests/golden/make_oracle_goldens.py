"""Write the oracle's results for the seeded square workloads.

Calls only the CPU oracle on the seeded workloads; the HIP path's tests
compare against the stored files.  Run from the repository root:

    python tests/golden/make_oracle_goldens.py 1   # 400 x 400, rank 10: tier A (dense Jacobi)
    python tests/golden/make_oracle_goldens.py 2   # 5000 x 5000, rank 10: tier B (Gram matrix)
    python tests/golden/make_oracle_goldens.py 2 60   # the same, X at iteration 60 (eps = 0)
    python tests/golden/make_oracle_goldens.py 3 40   # 10000 x 10000, rank 50: tier B, X at iteration 40

With a second argument k the run stops after k iterations with eps = 0, and
the file holds X^k: a fixed-iteration comparison point for trajectories
that amplify rounding differences (near the end of the 5000 x 5000 run the
rank of X flips between 10, 11 and 12, and two solvers that differ only in
rounding part ways).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workload  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main(cfg: int, kfix: int = 0):
    p = workload.config(cfg, seed=0)
    eps, maxiter = (0.0, kfix) if kfix > 0 else (p.eps, p.maxiter)
    t = time.time()
    if cfg == 1:
        out = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, eps,
                               maxiter, p.incr)
        tier = "A"
    else:
        out = oracle.svt_sparse(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, eps,
                                maxiter, p.incr,
                                progress=lambda k, r, res: print(f"  iteration {k}: rank {r}, "
                                                                 f"residual {res:.3e}", flush=True))
        tier = "B"
    dt = time.time() - t
    suffix = f"_k{kfix}" if kfix > 0 else ""
    path = os.path.join(HERE, f"oracle_config{cfg}{suffix}.npz")
    np.savez_compressed(path, U=out["U"], w=out["w"], V=out["V"], iters=out["iters"],
                        k0=out["k0"], sigma1=out["sigma1"], ranks=np.array(out["ranks"]),
                        s_hist=np.array(out["s_hist"]), residuals=np.array(out["residuals"]),
                        seconds=dt, tier=tier)
    print(f"wrote {path}: tier {tier}, {out['iters']} iterations, k0 {out['k0']}, {dt:.1f} s")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 1, int(sys.argv[2]) if len(sys.argv) > 2 else 0)
