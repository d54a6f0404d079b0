"""Benchmark of the SVT hot path on one MI355X.

A step is one full solve of Algorithm 1 (kick, SVT iterations to eps, factors
left on the device) on the 30000 x 30000, rank-10, |Omega| = 6 d_r workload
(the shape of Table 1's last row), with the problem already created (Omega,
values and index structures resident in HBM) before the timed region.

value = SVT iterations per second over the timed steps (loop iterations of
Algorithm 1, the kick's skipped steps not counted) of the plain FP64 solver
(the paper's precision); sampled entries/s = |Omega| x iterations/s.  The
mixed form (FP32 bulk, FP64 reductions) is reported beside it.  The roofline
object covers the headline's dominant kernel, timed with HIP events on the
solve's stream during the profiled steps.  The serving form reports
converged solves/s and latency percentiles over converged solves.  The CPU
baseline times the FP64 oracle on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
from paper_0810_3286_amd.svt import KERNEL_KINDS as KIND_NAMES  # noqa: E402
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
# the kernels and the launch configurations the solver picks for them
KERNEL_SRCS = [os.path.join(ROOT, "paper_0810_3286_amd", "csrc", f)
               for f in ("svt_kernels.hip", "svt_kernels.h", "svt_solver.cpp")]
# rocprofv3 kernel names of each timed kind (substring matches)
ROCPROF_NAMES = {
    "k_spmv": ("k_spmv",),
    "k_gs_update_pass1": ("k_gs_update<float, false>", "k_gs_update<double, false>"),
    "k_ritz": ("k_ritz",),
    "k_gather": ("k_gather",),
    "k_sample_update": ("k_sample_update",),
    "k_gs_update_pass2": ("k_gs_update<float, true>", "k_gs_update<double, true>"),
    "k_pending_reduce": ("k_pending_reduce",),
}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(kernel: str, workload: str, precision: str):
    """HBM bytes per launch from committed rocprofv3 counters, if they were
    taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        data = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if data.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    key = f"{workload}/{precision}/{kernel}"
    ent = data.get("kernels", {}).get(key)
    return None if ent is None else ent.get("bytes_per_launch")


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, seconds: float):
    """The CPU oracle as it stands, timed on the host on the same workload.

    At this size the oracle runs tier C: Algorithm 1 with the s_k largest
    singular triplets of each sparse iterate from SciPy's partial SVD
    (ARPACK), the sampled residual and the update in NumPy.  The sample is
    the kick plus the first SVT iterations, ended once the loop has run
    ``seconds``; the value is those loop iterations over the loop's wall time
    (the kick is reported apart, as on the GPU).
    """
    import oracle.krylov as ok
    try:
        from threadpoolctl import threadpool_info
        threads = max([i["num_threads"] for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:  # noqa: BLE001
        threads = int(os.environ.get("OMP_NUM_THREADS", "1"))
    t0 = time.perf_counter()
    out = ok.svt_krylov(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr,
                        max_seconds=seconds)
    t_all = time.perf_counter() - t0
    loop_s = float(np.sum(out["seconds"]))
    iters = len(out["seconds"])
    ips = iters / loop_s
    log(f"[bench] cpu baseline: {iters} oracle iterations in {loop_s:.1f} s (+ kick {t_all - loop_s:.1f} s)")
    return {
        "value": ips,
        "unit": "SVT iters/s",
        "sampled_entries_per_s": ips * p.nnz,
        "cores": threads,
        "cpu_model": _cpu_model(),
        "host_cpus": os.cpu_count(),
        "kind": "oracle",
        "sample": (f"the FP64 oracle (tier C: Algorithm 1 with SciPy's ARPACK partial SVD of each sparse "
                   f"iterate) on the same {p.m} x {p.n} workload: the kick ({t_all - loop_s:.1f} s) and SVT "
                   f"iterations 1..{iters}, timed ({loop_s:.1f} s of loop, {loop_s / iters:.2f} s per "
                   f"iteration); BLAS threads {threads}, the sparse products single-threaded"),
        "oracle_ranks": out["ranks"],
    }


def _pmc_per_kernel(run_dir: str, counter: str):
    """Mean counter value (KiB) per dispatch of each kernel name in a
    rocprofv3 --pmc CSV run directory."""
    import csv
    import glob
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {run_dir}")
    tot, cnt = {}, {}
    for f in files:
        for row in csv.DictReader(open(f)):
            if row["Counter_Name"] != counter:
                continue
            k = row["Kernel_Name"]
            tot[k] = tot.get(k, 0.0) + float(row["Counter_Value"])
            cnt[k] = cnt.get(k, 0) + 1
    return {k: (tot[k] / cnt[k], cnt[k]) for k in tot}


def traffic_summary(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_mib, workload, precision,
                    algorithmic):
    """HBM bytes per launch of each timed kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE), each scaled by what the same counter reads for
    the runtime's copy kernel moving copy_mib MiB; writes the committed
    traffic file and prints a text summary."""
    nbytes = float(copy_mib << 20)
    cf = _pmc_per_kernel(copy_fetch_dir, "FETCH_SIZE")
    cw = _pmc_per_kernel(copy_write_dir, "WRITE_SIZE")

    def copy_mean(d):
        ent = [v for k, v in d.items() if "copyBuffer" in k]
        if not ent:
            raise SystemExit("no copy-kernel dispatch in the calibration run")
        # the largest mean is the copy of the full buffer
        return max(e[0] for e in ent)
    f_fetch = nbytes / (copy_mean(cf) * 1024.0)
    f_write = nbytes / (copy_mean(cw) * 1024.0)
    fe = _pmc_per_kernel(fetch_dir, "FETCH_SIZE")
    wr = _pmc_per_kernel(write_dir, "WRITE_SIZE")
    out = {"kernel_source_sha256_16": kernel_source_hash(), "copy_mib": copy_mib,
           "fetch_factor": f_fetch, "write_factor": f_write, "kernels": {}}
    lines = [f"copy calibration ({copy_mib} MiB): FETCH_SIZE x {f_fetch:.3f}, WRITE_SIZE x {f_write:.3f}",
             f"{'kernel':<20} {'dispatches':>10} {'fetch MB':>10} {'write MB':>10} {'HBM MB':>10} {'alg MB':>10}"]
    for kind, pats in ROCPROF_NAMES.items():
        def agg(d):
            n_ = sum(v[1] for k, v in d.items() if any(pt in k for pt in pats))
            s_ = sum(v[0] * v[1] for k, v in d.items() if any(pt in k for pt in pats))
            return (s_ / n_ if n_ else 0.0), n_
        fkib, nf = agg(fe)
        wkib, nw = agg(wr)
        if nf == 0:
            continue
        hbm = fkib * 1024.0 * f_fetch + wkib * 1024.0 * f_write
        key = f"{workload}/{precision}/{kind}"
        alg = algorithmic.get(kind)
        out["kernels"][key] = {"dispatches": nf, "fetch_bytes_per_launch": fkib * 1024.0 * f_fetch,
                               "write_bytes_per_launch": wkib * 1024.0 * f_write, "bytes_per_launch": hbm,
                               "algorithmic_bytes_per_launch": alg}
        lines.append(f"{kind:<20} {nf:>10d} {fkib * 1024 * f_fetch / 1e6:>10.3f} {wkib * 1024 * f_write / 1e6:>10.3f} "
                     f"{hbm / 1e6:>10.3f} {(alg or 0) / 1e6:>10.3f}")
    old = {}
    if os.path.exists(TRAFFIC_FILE):
        try:
            old = json.load(open(TRAFFIC_FILE))
        except ValueError:
            old = {}
    if old.get("kernel_source_sha256_16") == out["kernel_source_sha256_16"]:
        merged = dict(old.get("kernels", {}))
        merged.update(out["kernels"])
        out["kernels"] = merged
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print("\n".join(lines))


def table2_runs(precisions=("fp64", "mixed"), seed: int = 7) -> dict:
    """Table 2's shapes (Section 5.2.1): n = 1000, (r, |Omega| / d_r) = (10, 6),
    (50, 4), (100, 3), noise ratios 1e-2, 1e-1, 1, each solved once with the
    eq. (5.10) stop (the paper averages five runs).  Per case: iterations,
    seconds (from svt_create's return to the factors, warm), relative error
    against the truth, and the paper's iterations and error for reference."""
    import numpy as np
    import workload
    from paper_0810_3286_amd import svt as B
    paper = {(10, 1e-2): (51, 0.78e-2), (50, 1e-2): (48, 0.95e-2), (100, 1e-2): (50, 1.13e-2),
             (10, 1e-1): (19, 0.72e-1), (50, 1e-1): (17, 0.89e-1), (100, 1e-1): (17, 1.01e-1),
             (10, 1.0): (3, 0.52), (50, 1.0): (3, 0.63), (100, 1.0): (3, 0.69)}
    out = []
    for prec in precisions:
        for ratio in workload.TABLE2_NOISE_RATIOS:
            for r, c in workload.TABLE2_RANK_OVERSAMPLING:
                p = workload.noisy_lowrank(1000, r, c, ratio, seed)
                prm = B.svt_params_default(p.m, p.n, len(p.vals))
                prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, p.delta, p.eps, p.maxiter, p.incr
                prm.stop_rule = B.SVT_STOP_NOISY
                prm.noise_sigma = p.noise_sigma
                prm.precision = B.SVT_FP64 if prec == "fp64" else B.SVT_MIXED
                h = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
                try:
                    B.svt_solve(h)   # warm-up: the library's first-call costs
                    t0 = time.perf_counter()
                    st, info = B.svt_solve(h)
                    U, w, V = B.svt_factors(h, p.m, p.n)
                    dt = time.perf_counter() - t0
                finally:
                    B.svt_destroy(h)
                M = p.ML @ p.MR.T
                rel = float(np.linalg.norm(U @ V.T - M) / np.linalg.norm(M))
                pi, pe = paper[(r, ratio)]
                out.append({"precision": prec, "noise_ratio": ratio, "rank": r, "nnz_over_dr": c,
                            "iters": int(info.iters), "seconds": dt, "rel_error": rel,
                            "paper_iters": pi, "paper_rel_error": pe, "status": int(st)})
                log(f"[bench] table2 {prec} ratio {ratio:g} rank {r}: {info.iters} iterations, "
                    f"{dt:.3f} s, relative error {rel:.3e} (paper: {pi}, {pe:.2e})")
    return {"table2": out}


def _timed_solve(B, h):
    B.svt_solve(h)   # warm-up: the library's first-call costs
    t0 = time.perf_counter()
    st, info = B.svt_solve(h)
    return st, info, time.perf_counter() - t0


def dantzig_runs(seed: int = 0) -> dict:
    """Section 5.2.2 (Figure 3): n = 1000, r = 10, |Omega| = 5 d_r, noise
    sigma = 0.1 x the mean |M_ij| on Omega, constraints |X_ij - B_ij| <= sigma
    on Omega (the Dantzig-selector iteration, eq. (3.10)).  Runs: the paper's
    step delta = 1.2 / p (300 iterations), half that step with the eq. (5.10)
    stop, in both precisions, and Algorithm 1 on the noiseless data."""
    import numpy as np
    import workload
    from paper_0810_3286_amd import svt as B
    from tests.helpers import rel_diff_factored
    p = workload.dantzig_fig3(seed=seed)
    out = {"noise_ratio": float(np.linalg.norm(p.vals - p.clean) / np.linalg.norm(p.clean)), "runs": []}

    def run(label, vals, precision, delta, ds, maxiter, noisy):
        prm = B.svt_params_default(p.m, p.n, p.nnz)
        prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, delta, p.eps, maxiter, p.incr
        prm.precision = precision
        if ds:
            prm.constraint = B.SVT_CONSTRAINT_INEQUALITY
            prm.ineq_tol = p.noise_sigma
        if noisy:
            prm.stop_rule = B.SVT_STOP_NOISY
            prm.noise_sigma = p.noise_sigma
        h = B.svt_create(p.m, p.n, p.rows, p.cols, vals, prm)
        try:
            st, info, dt = _timed_solve(B, h)
            U, w, V = B.svt_factors(h, p.m, p.n)
            hist = B.svt_history(h)
        finally:
            B.svt_destroy(h)
        rec = {"run": label, "precision": "fp64" if precision == B.SVT_FP64 else "mixed",
               "status": B.svt_status_string(st), "iters": int(info.iters), "seconds": dt,
               "final_rank": int(info.rank), "max_rank": int(max(hist["ranks"])) if len(hist["ranks"]) else 0,
               "rel_error_vs_truth": rel_diff_factored(U, V, p.ML, p.MR)}
        out["runs"].append(rec)
        log(f"[bench] dantzig {rec}")

    for prec in (B.SVT_FP64, B.SVT_MIXED):
        run("inequality, delta = 0.6 / p, eq. (5.10) stop", p.vals, prec, 0.5 * p.delta, True, p.maxiter, True)
    run("inequality, delta = 1.2 / p (the paper's step)", p.vals, B.SVT_FP64, p.delta, True, 300, False)
    run("equality, noiseless data", p.clean, B.SVT_FP64, p.delta, False, p.maxiter, False)
    return {"dantzig_fig3": out}


def sensing_runs(seed: int = 0) -> dict:
    """A general linear operator (Section 3.1): 3000 x 3000, rank 10, p =
    8 d_r measurements of 4 entries each; both precisions."""
    import workload
    from paper_0810_3286_amd import svt as B
    from tests.helpers import rel_diff_factored
    q = workload.sparse_sensing(3000, 3000, 10, 8 * 10 * (6000 - 10), 4, seed=seed)
    out = []
    for prec in (B.SVT_FP64, B.SVT_MIXED):
        prm = B.svt_params_default(q.m, q.n, q.p)
        prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = q.tau, q.delta, q.eps, q.maxiter, q.incr
        prm.precision = prec
        h = B.svt_create_sensing(q.m, q.n, q.srows, q.scols, q.gptr, q.gidx, q.gval, q.b, prm)
        try:
            st, info, dt = _timed_solve(B, h)
            U, w, V = B.svt_factors(h, q.m, q.n)
        finally:
            B.svt_destroy(h)
        rec = {"precision": "fp64" if prec == B.SVT_FP64 else "mixed", "status": B.svt_status_string(st),
               "iters": int(info.iters), "seconds": dt, "svt_iters_per_s": info.iters / dt,
               "final_rank": int(info.rank), "rel_error_vs_truth": rel_diff_factored(U, V, q.ML, q.MR),
               "measurements": q.p, "support": int(q.srows.shape[0])}
        out.append(rec)
        log(f"[bench] sensing {rec}")
    return {"sensing": out}


def randomized_runs(maxiter: int = 200) -> dict:
    """D_tau by the randomised range finder (Section 6) against the
    Lanczos partial SVD on 400^2 (rank 10, 6 d_r) and 5000^2 (rank 10,
    5 d_r), FP64: status, iterations, the smallest residual reached and the
    error against the truth, for 1, 2 and 4 power iterations."""
    import workload
    from paper_0810_3286_amd import svt as B
    from tests.helpers import rel_diff_factored
    out = []
    for cfg in (1, 2):
        p = workload.config(cfg)
        for method, power in ((B.SVT_SVD_LANCZOS, 0), (B.SVT_SVD_RANDOMIZED, 1), (B.SVT_SVD_RANDOMIZED, 2),
                              (B.SVT_SVD_RANDOMIZED, 4)):
            prm = B.svt_params_default(p.m, p.n, p.nnz)
            prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, p.delta, p.eps, maxiter, p.incr
            prm.svd_method = method
            prm.rsvd_power = power
            h = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
            try:
                st, info, dt = _timed_solve(B, h)
                U, w, V = B.svt_factors(h, p.m, p.n)
                hist = B.svt_history(h)
            finally:
                B.svt_destroy(h)
            rec = {"config": f"{p.m}x{p.n} r{p.r}", "method": "lanczos" if method == B.SVT_SVD_LANCZOS else
                   f"randomized q={power}", "status": B.svt_status_string(st), "iters": int(info.iters),
                   "seconds": dt, "svt_iters_per_s": info.iters / dt, "min_residual": float(np.min(hist["residuals"])),
                   "rel_error_vs_truth": rel_diff_factored(U, V, p.ML, p.MR), "final_rank": int(info.rank)}
            out.append(rec)
            log(f"[bench] randomized {rec}")
    return {"randomized_svd": out}


def copy_calibration(mib: int, reps: int = 3):
    """Device-to-device copies of a known size through the HIP runtime's copy
    kernel: under rocprofv3 --pmc its FETCH_SIZE / WRITE_SIZE per dispatch,
    divided by the bytes copied, calibrate the counters."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    nbytes = mib << 20
    src, dst = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(src), ctypes.c_size_t(nbytes)) == 0
    assert hip.hipMalloc(ctypes.byref(dst), ctypes.c_size_t(nbytes)) == 0
    assert hip.hipMemset(src, 1, ctypes.c_size_t(nbytes)) == 0
    for _ in range(reps):
        assert hip.hipMemcpy(dst, src, ctypes.c_size_t(nbytes), 3) == 0  # device to device
    assert hip.hipDeviceSynchronize() == 0
    hip.hipFree(src)
    hip.hipFree(dst)
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}), flush=True)


def serving_bench(n_req: int, slots: int, budget_gib: float, precision: int, seed: int = 0,
                  load_fracs=(0.7, 0.9), mix: str = "baseline", step_cap: int = 512,
                  noise_frac: float = 0.0, open_loop: bool = True, min_rows: int = 0):
    """Serving form on a stream of mixed completion requests.

    mix "baseline": m, n uniform in [500, 8000] (rectangular), r in
    {5, 10, 20, 50}, |Omega| = c r (m + n - r) with c uniform in [3, 6].
    mix "table1": m, n uniform in [1000, 8000] (aspect ratio at most 1.5),
    (r, c) drawn from Table 1's pairs (10, 6), (50, 5), (100, 4).
    Both: tau = 5 sqrt(m n), delta = 1.2 m n / |Omega|, eps = 1e-4, maxiter
    500; each request's bidiagonalisation is capped at step_cap steps (a
    request that needs more ends with SVT_ELANCZOS), the server's stall
    bound ends a request whose residual sets no new minimum for 20 iterations
    (SVT_STALLED) and its degrees-of-freedom bound one whose iterate's rank
    has more degrees of freedom than the request has observations
    (SVT_UNDERDETERMINED), so a request outside the method's regime holds its
    slot for a bounded time.  noise_frac: that share of the requests carries
    N(0, 0.01^2) noise on its observations and stops by eq. (5.10) with
    sigma = 0.01 and eps = 0.1 (the others as above).
    Closed loop (all requests at t = 0) gives the capacity C in requests/s;
    open loops with Poisson arrivals at each of load_fracs times C (fresh
    requests of the same stream for each) give the latency (arrival to
    completion).  Solves/s and the latency percentiles count converged solves
    (SVT_OK) only; the status split and the latencies of the other requests
    are reported beside them."""
    import threading
    import workload
    from paper_0810_3286_amd import svt as B
    nruns = 1 + (len(load_fracs) if open_loop else 0)
    if mix == "table1":
        trace = workload.serving_trace(nruns * n_req, seed=seed, rate=1.0, mn_range=(1000, 8000),
                                       pairs=workload.TABLE1_RANK_OVERSAMPLING, max_aspect=1.5,
                                       noise_frac=noise_frac)
    else:
        trace = workload.serving_trace(nruns * n_req, seed=seed, rate=1.0, noise_frac=noise_frac)
    probs = []
    for _, sp in trace:
        probs.append(workload.gaussian_lowrank(sp["m"], sp["n"], sp["r"], sp["nnz"], sp["seed"],
                                               noise_sigma=sp["noise_sigma"], maxiter=500))
        log(f"[bench] serving request {len(probs) - 1} generated ({sp['m']} x {sp['n']}, r {sp['r']}, "
            f"|Omega| {sp['nnz']}{', noisy' if sp['noise_sigma'] > 0 else ''})")

    def params(p):
        prm = B.svt_params_default(p.m, p.n, p.nnz)
        prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, p.delta, p.eps, p.maxiter, p.incr
        prm.precision = precision
        prm.lanczos_maxsteps = step_cap
        prm.min_block_rows = min_rows      # 0: the server's choice
        if p.noise_sigma > 0:
            prm.stop_rule = B.SVT_STOP_NOISY
            prm.noise_sigma = p.noise_sigma
            prm.eps = 0.1
        return prm

    pct = (lambda a, q: float(np.percentile(a, q)) if len(a) else None)
    budget = int(budget_gib * (1 << 30))
    srv = B.svt_server_create(budget, slots)
    statuses = []

    def run_open(frac, openp, capacity, rseed):
        rate = frac * capacity
        rng = np.random.default_rng(rseed)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, len(openp)))
        tix = [None] * len(openp)

        def submitter():
            base = time.perf_counter()
            for i, p in enumerate(openp):
                dt = arrivals[i] - (time.perf_counter() - base)
                if dt > 0:
                    time.sleep(dt)
                tix[i] = B.svt_submit(srv, p.m, p.n, p.rows, p.cols, p.vals, params(p))
                log(f"[bench] serving open loop {frac}: request {i} submitted")

        t1 = time.perf_counter()
        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        lat, lat_failed = [], []
        for i, p in enumerate(openp):
            st, info = B.svt_wait(srv, tix[i])
            _, _, _, _, times = B.svt_result(srv, tix[i], p.m, p.n)
            li = times[2] - times[0]
            (lat if st == B.SVT_OK else lat_failed).append(li)
            statuses.append(st)
            B.svt_release(srv, tix[i])
            log(f"[bench] serving open loop {frac}: request {i} done (status {st}, latency {li:.2f} s)")
        t_open = time.perf_counter() - t1
        return {"load_frac": frac, "rate_per_s": rate, "solves_per_s": len(lat) / t_open,
                "converged": len(lat), "p50_latency_s": pct(lat, 50), "p99_latency_s": pct(lat, 99),
                "failed_latency_s": sorted(float(x) for x in lat_failed)}

    try:
        closed = probs[:n_req]
        t0 = time.perf_counter()
        tickets = [B.svt_submit(srv, p.m, p.n, p.rows, p.cols, p.vals, params(p)) for p in closed]
        iters = 0
        entries = 0
        spmv_bytes = 0.0
        vbytes = 4.0 if precision == B.SVT_MIXED else 8.0
        closed_ok = 0
        for i, t in enumerate(tickets):
            st, info = B.svt_wait(srv, t)
            iters += info.iters
            entries += info.iters * closed[i].nnz
            # the sparse products' algorithmic bytes: two per bidiagonalisation
            # step, each streaming every stored entry (value and 16-bit index)
            spmv_bytes += 2.0 * info.gkl_steps * closed[i].nnz * (vbytes + 2.0)
            statuses.append(st)
            closed_ok += int(st == B.SVT_OK)
            B.svt_release(srv, t)
            log(f"[bench] serving closed loop: request {i} done (status {st}, {info.iters} iterations)")
        t_closed = time.perf_counter() - t0
        capacity = n_req / t_closed
        log(f"[bench] serving closed loop: {n_req} requests ({closed_ok} converged) in {t_closed:.2f} s")
        opens = []
        if open_loop:
            for q, frac in enumerate(load_fracs):
                opens.append(run_open(frac, probs[(q + 1) * n_req:(q + 2) * n_req], capacity, seed + 1 + q))
        stats = B.svt_server_stats(srv)
    finally:
        B.svt_server_destroy(srv)
    out = {
        "requests_per_run": n_req, "slots": slots, "budget_gib": budget_gib,
        "precision": "mixed" if precision == B.SVT_MIXED else "fp64",
        "noisy_share": noise_frac,
        # converged solves (SVT_OK) only; requests that ended otherwise are
        # counted apart
        "closed_loop_solves_per_s": closed_ok / t_closed,
        "closed_loop_converged": closed_ok,
        "closed_loop_requests_per_s": capacity,
        "closed_loop_svt_iters_per_s": iters / t_closed,
        "closed_loop_sampled_entries_per_s": entries / t_closed,
        # aggregate HBM rate of the sparse products over the closed loop
        # (their stored entries only), as a fraction of the 8 TB/s peak
        "closed_loop_spmv_hbm_frac": spmv_bytes / t_closed / 8e12,
        "mix": mix, "step_cap": step_cap,
        # the server's defaults for what the requests leave unset: the stall
        # window, the degrees-of-freedom bound (multiples of |Omega|) and the
        # row-block minimum (min_rows, when 0)
        "server_defaults": {"stall_window": 20, "dof_bound": 1.0, "min_block_rows": 64},
        "status_counts": {B.svt_status_string(k): int(v) for k, v in
                          zip(*np.unique(np.array(statuses), return_counts=True))},
        "max_running": stats["max_running"], "peak_admitted_gib": stats["peak_bytes"] / (1 << 30),
    }
    if opens:
        o = opens[0]
        out.update({"open_loop_rate_per_s": o["rate_per_s"], "open_loop_solves_per_s": o["solves_per_s"],
                    "open_loop_converged": o["converged"], "p50_latency_s": o["p50_latency_s"],
                    "p99_latency_s": o["p99_latency_s"], "failed_latency_s": o["failed_latency_s"],
                    "open_loops": opens})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="the headline form (fp64: the paper's precision); the other form is "
                         "reported beside it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--profile-steps", type=int, default=1)
    ap.add_argument("--spmv-mode", type=int, default=0,
                    help="0 or 2: x staged in LDS (column segments when needed), 1: gathered")
    ap.add_argument("--reorth-eta", type=float, default=None,
                    help="partial reorthogonalisation level, a multiple of sqrt(unit roundoff) "
                         "(0: every vector orthogonalised; default: the library's automatic level, "
                         "reported as -1)")
    ap.add_argument("--min-rows", type=int, default=0,
                    help="min_block_rows of the headline solve (0: the library default)")
    ap.add_argument("--serving-requests", type=int, default=64,
                    help="requests per serving run (closed loop, each open loop, noisy run)")
    ap.add_argument("--serving-slots", type=int, default=8)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-mix", choices=["baseline", "table1"], default="baseline")
    ap.add_argument("--serving-step-cap", type=int, default=512)
    ap.add_argument("--serving-min-rows", type=int, default=0,
                    help="min_block_rows of the served requests (0: the server's default)")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the run of the other precision (mixed beside an fp64 headline, or fp64 "
                         "beside a mixed one)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (counter calibration)")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                         "COPY_WRITE_DIR"),
                    help="write the HBM traffic file from rocprofv3 --pmc runs of this bench "
                         "(FETCH_SIZE, WRITE_SIZE) and of --copy-calibration (same two counters); "
                         "needs --traffic-mib and --traffic-bench-json")
    ap.add_argument("--table2", action="store_true",
                    help="run Table 2's noisy-data shapes (n = 1000) and print their results instead")
    ap.add_argument("--dantzig", action="store_true",
                    help="run Figure 3's inequality-constrained (Dantzig selector) workload and print its results")
    ap.add_argument("--sensing", action="store_true",
                    help="run a general-linear-operator (sparse measurement) workload and print its results")
    ap.add_argument("--randomized", action="store_true",
                    help="compare the randomised partial SVD with the Lanczos one and print the results")
    ap.add_argument("--traffic-mib", type=int, default=256)
    ap.add_argument("--traffic-bench-json", help="the JSON line of the counted bench run")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.traffic_summary:
        line = open(args.traffic_bench_json).read().strip().splitlines()[-1]
        bj = json.loads(line)
        alg = {k: v.get("bytes_per_launch") for k, v in bj["kernels"].items()}
        traffic_summary(*args.traffic_summary, args.traffic_mib, bj["config"]["workload"],
                        bj["config"]["precision"], alg)
        return

    if args.table2:
        print(json.dumps(table2_runs()), flush=True)
        return
    if args.dantzig:
        print(json.dumps(dantzig_runs()), flush=True)
        return
    if args.sensing:
        print(json.dumps(sensing_runs()), flush=True)
        return
    if args.randomized:
        print(json.dumps(randomized_runs()), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the SVT solve here runs on a single MI355X and "
              "no multi-GPU path is built (request sharding across GPUs is a design note only).",
              file=sys.stderr)
        sys.exit(2)

    import workload
    from paper_0810_3286_amd import svt as B

    log(f"[bench] generating workload config {args.config}")
    p = workload.config(args.config, seed=0)
    prec = B.SVT_MIXED if args.precision == "mixed" else B.SVT_FP64
    wl_name = p.name

    eta_used = [0.0]

    def make(profile):
        prm = B.svt_params_default(p.m, p.n, p.nnz)
        prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, p.delta, p.eps, p.maxiter, p.incr
        prm.precision = prec
        prm.profile = 1 if profile else 0
        prm.spmv_mode = args.spmv_mode
        prm.min_block_rows = args.min_rows
        if args.reorth_eta is not None:
            prm.reorth_eta = args.reorth_eta
        eta_used[0] = prm.reorth_eta
        return B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)

    log("[bench] svt_create")
    t0 = time.perf_counter()
    h = make(False)
    t_create = time.perf_counter() - t0
    infos = []
    try:
        for i in range(args.warmup):
            log(f"[bench] warmup solve {i}")
            st, info = B.svt_solve(h)
        log(f"[bench] timed solves x{args.steps}")
        t0 = time.perf_counter()
        for i in range(args.steps):
            st, info = B.svt_solve(h)
            infos.append(info.as_dict())
        t_total = time.perf_counter() - t0
        U, w, V = B.svt_factors(h, p.m, p.n)
        hist = B.svt_history(h)
        reorth = B.svt_reorth_stats(h)
    finally:
        B.svt_destroy(h)

    iters = sum(i["iters"] for i in infos)
    loop_s = sum(i["t_solve_s"] for i in infos)
    kick_s = sum(i["t_kick_s"] for i in infos)
    iters_per_s = iters / t_total
    from tests.helpers import rel_diff_factored
    relerr = rel_diff_factored(U, V, p.ML, p.MR)

    # profiled steps: per-kernel-class HIP event timing on the solve's stream
    log(f"[bench] profiled solves x{args.profile_steps}")
    hp = make(True)
    try:
        kstats = {}
        for i in range(args.profile_steps):
            B.svt_solve(hp)
            for kind in KIND_NAMES:
                n_, ms_, by_ = B.svt_kernel_stats(hp, kind)
                a = kstats.setdefault(kind, [0, 0.0, 0.0])
                a[0] += n_; a[1] += ms_; a[2] += by_
    finally:
        B.svt_destroy(hp)
    if not kstats:
        kstats = {0: [0, 0.0, 0.0]}
    dom = max(kstats, key=lambda k: kstats[k][1])
    n_l, ms_l, by_l = kstats[dom]
    avg_s = ms_l / 1e3 / max(n_l, 1)
    bytes_per_launch = by_l / max(n_l, 1)
    achieved = bytes_per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    traffic = measured_traffic(KIND_NAMES[dom], wl_name, args.precision)

    out = {
        "metric": "SVT iters/s + sampled entries/s at n=30k r=10; solves/s, p99 latency",
        "value": iters_per_s,
        "unit": "SVT iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == B.SVT_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl_name, "m": p.m, "n": p.n, "rank": p.r, "nnz": p.nnz,
                   "tau": p.tau, "delta": p.delta, "eps": p.eps,
                   "precision": args.precision, "parallelism": "single-gpu"},
        "sampled_entries_per_s": iters_per_s * p.nnz,
        "solves_per_s_30k": args.steps / t_total,
        "iters_per_solve": iters / args.steps,
        "loop_iters_per_s": iters / loop_s,
        "kick_s_per_solve": kick_s / args.steps,
        "setup_s": t_create,
        "rel_error_vs_truth": relerr,
        "final_rank": int(hist["ranks"][-1]) if len(hist["ranks"]) else 0,
        "gkl_steps_per_iter": float(np.mean(hist["gkl_steps"])) if len(hist["gkl_steps"]) else 0.0,
        "reorth": {"eta": eta_used[0], "vectors": reorth[0],
                   "orthogonalised": reorth[1], "two_pass_restarts": reorth[2],
                   "partial_fallbacks": reorth[3]},
        "kernels": {KIND_NAMES[k]: {"launches": v[0], "ms": v[1],
                                    "avg_us": v[1] * 1e3 / max(v[0], 1),
                                    "bytes_per_launch": v[2] / max(v[0], 1),
                                    "GBps": (v[2] / (v[1] / 1e3) / 1e9) if v[1] > 0 else 0.0}
                    for k, v in kstats.items()},
        "roofline": {"kernel": KIND_NAMES[dom], "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": avg_s * 1e6},
    }
    if not args.no_other:
        # the other precision on the same workload: the mixed form beside the
        # plain FP64 solver (or the FP64 solver beside a mixed headline)
        other = "mixed" if args.precision == "fp64" else "fp64"
        prm = B.svt_params_default(p.m, p.n, p.nnz)
        prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, p.delta, p.eps, p.maxiter, p.incr
        prm.precision = B.SVT_MIXED if other == "mixed" else B.SVT_FP64
        if args.reorth_eta is not None:
            prm.reorth_eta = args.reorth_eta
        prm.spmv_mode = args.spmv_mode
        prm.min_block_rows = args.min_rows
        ho = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
        try:
            log(f"[bench] {other} solves")
            for _ in range(max(args.warmup, 1)):
                B.svt_solve(ho)
            t0 = time.perf_counter()
            ito = 0
            for _ in range(args.steps):
                _, inf = B.svt_solve(ho)
                ito += inf.iters
            to = time.perf_counter() - t0
            Uo, _, Vo = B.svt_factors(ho, p.m, p.n)
            ro = B.svt_reorth_stats(ho)
        finally:
            B.svt_destroy(ho)
        out[other] = {"svt_iters_per_s": ito / to, "sampled_entries_per_s": ito / to * p.nnz,
                      "iters_per_solve": ito / args.steps, "ms_per_step": to / args.steps * 1e3,
                      "dtype": "f64" if other == "fp64" else "f32+f64",
                      "rel_error_vs_truth": rel_diff_factored(Uo, Vo, p.ML, p.MR),
                      "rel_diff_vs_headline": rel_diff_factored(Uo, Vo, U, V),
                      "reorth": {"eta": prm.reorth_eta, "vectors": ro[0], "orthogonalised": ro[1],
                                 "partial_fallbacks": ro[3]}}
    if not args.no_serving:
        log("[bench] serving stream")
        # the serving form runs mixed-precision solves (its workload's definition)
        out["serving"] = serving_bench(args.serving_requests, args.serving_slots, 64.0, B.SVT_MIXED,
                                       mix=args.serving_mix, step_cap=args.serving_step_cap,
                                       min_rows=args.serving_min_rows)
        # converged solves only (the status split is in "serving")
        out["solves_per_s"] = out["serving"]["closed_loop_solves_per_s"]
        out["p99_latency_s"] = out["serving"]["p99_latency_s"]
        # the same stream with half of the requests noisy (eq. (5.10) stop),
        # closed loop
        out["serving_noisy"] = serving_bench(args.serving_requests, args.serving_slots, 64.0, B.SVT_MIXED,
                                             mix=args.serving_mix, step_cap=args.serving_step_cap,
                                             noise_frac=0.5, open_loop=False, min_rows=args.serving_min_rows)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
