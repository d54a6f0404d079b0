"""Write the oracle's results for the 400 x 400 workload (rank 10, |Omega| = 6 d_r).

Calls only the CPU oracle (``oracle.svt_dense``) on the seeded workload; the
HIP path's tests compare against the stored file.  Run from the repository
root: ``python tests/golden/make_oracle_goldens.py``.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workload  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_config1.npz")


def main():
    p = workload.config(1, seed=0)
    t = time.time()
    out = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps,
                           p.maxiter, p.incr)
    dt = time.time() - t
    np.savez_compressed(OUT, U=out["U"], w=out["w"], V=out["V"], iters=out["iters"],
                        k0=out["k0"], sigma1=out["sigma1"], ranks=np.array(out["ranks"]),
                        s_hist=np.array(out["s_hist"]), residuals=np.array(out["residuals"]),
                        seconds=dt)
    print(f"wrote {OUT}: {out['iters']} iterations, k0 {out['k0']}, {dt:.1f} s")


if __name__ == "__main__":
    main()
