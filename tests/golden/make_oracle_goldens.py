"""Write the oracle's results for the seeded square workloads.

Calls only the CPU oracle on the seeded workloads; the HIP path's tests
compare against the stored files.  Run from the repository root:

    python tests/golden/make_oracle_goldens.py 1   # 400 x 400, rank 10: tier A (dense Jacobi)
    python tests/golden/make_oracle_goldens.py 2   # 5000 x 5000, rank 10: tier B (Gram matrix)
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


def main(cfg: int):
    p = workload.config(cfg, seed=0)
    t = time.time()
    if cfg == 1:
        out = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps,
                               p.maxiter, p.incr)
        tier = "A"
    else:
        out = oracle.svt_sparse(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps,
                                p.maxiter, p.incr,
                                progress=lambda k, r, res: print(f"  iteration {k}: rank {r}, "
                                                                 f"residual {res:.3e}", flush=True))
        tier = "B"
    dt = time.time() - t
    path = os.path.join(HERE, f"oracle_config{cfg}.npz")
    np.savez_compressed(path, U=out["U"], w=out["w"], V=out["V"], iters=out["iters"],
                        k0=out["k0"], sigma1=out["sigma1"], ranks=np.array(out["ranks"]),
                        s_hist=np.array(out["s_hist"]), residuals=np.array(out["residuals"]),
                        seconds=dt, tier=tier)
    print(f"wrote {path}: tier {tier}, {out['iters']} iterations, k0 {out['k0']}, {dt:.1f} s")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 1)
