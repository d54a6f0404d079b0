"""How far the oracle's own complete run at 5000 x 5000, rank 10, |Omega| =
5 d_r moves when its inputs or its arithmetic change only by rounding.

Calls only the CPU oracle (tier C) on the seeded workload, several times:

  * "base": the workload as generated;
  * "ulp<s>": every observed value moved by one unit in the last place, up or
    down at random (seed s);
  * "start<s>": the partial SVD's start vectors drawn from another seed (the
    converged triplets are the same up to rounding).

For each run it stores the iteration count, the rank and residual history
and the final X's distance to the base run's, so a test can state the
spread of the stop iteration and the growth of the difference with the
iteration count as properties of the method on this workload, not of any
solver under test.  Run from the repository root (about 3 minutes per run on
the container's host; runs in parallel processes):

    python tests/golden/make_rounding_spread.py
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

HERE = os.path.dirname(os.path.abspath(__file__))
RUNS = ["base"] + [f"ulp{i}" for i in range(1, 17)] + [f"start{i}" for i in range(1, 5)]


def one(name):
    os.environ.setdefault("OMP_NUM_THREADS", "2")
    import workload
    from oracle.krylov import svt_krylov
    p = workload.config(2, seed=0)
    vals = p.vals.copy()
    seed = 0
    if name.startswith("ulp"):
        rng = np.random.default_rng(int(name[3:]))
        up = rng.integers(0, 2, size=vals.shape[0]).astype(bool)
        vals = np.where(up, np.nextafter(vals, np.inf), np.nextafter(vals, -np.inf))
    elif name.startswith("start"):
        seed = 1000 * int(name[5:])
    out = svt_krylov(p.m, p.n, p.rows, p.cols, vals, p.tau, p.delta, p.eps, p.maxiter, p.incr, seed=seed)
    print(f"{name}: {out['iters']} iterations, final rank {out['ranks'][-1]}", flush=True)
    return name, out


def main():
    with ProcessPoolExecutor(max_workers=4) as ex:
        res = dict(ex.map(one, RUNS))
    from tests.helpers import rel_diff_factored
    base = res["base"]
    L = max(len(r["residuals"]) for r in res.values())
    iters = np.array([res[n]["iters"] for n in RUNS])
    resid = np.full((len(RUNS), L), np.nan)
    ranks = np.full((len(RUNS), L), -1)
    for i, n in enumerate(RUNS):
        resid[i, :len(res[n]["residuals"])] = res[n]["residuals"]
        ranks[i, :len(res[n]["ranks"])] = res[n]["ranks"]
    xdiff = np.array([rel_diff_factored(res[n]["U"], res[n]["V"], base["U"], base["V"]) for n in RUNS])
    np.savez_compressed(os.path.join(HERE, "oracle_config2_spread.npz"), runs=np.array(RUNS), iters=iters,
                        residuals=resid, ranks=ranks, x_rel_diff_vs_base=xdiff)
    print("iterations:", dict(zip(RUNS, iters.tolist())))
    print("final X vs base:", dict(zip(RUNS, xdiff.tolist())))


if __name__ == "__main__":
    main()
