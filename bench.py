"""Benchmark of the SVT hot path on one MI355X.

A step is one full solve of Algorithm 1 (kick, SVT iterations to eps, factors
left on the device) on the 30000 x 30000, rank-10, |Omega| = 6 d_r workload
(the shape of Table 1's last row), with the problem already created (Omega,
values and index structures resident in HBM) before the timed region.

value = SVT iterations per second over the timed steps (loop iterations of
Algorithm 1, the kick's skipped steps not counted); sampled entries/s =
|Omega| x iterations/s.  The roofline object covers the dominant kernel,
timed with HIP events on the solve's stream during the profiled steps.
The CPU baseline times the FP64 oracle on the host.
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
KERNEL_SRC = os.path.join(ROOT, "paper_0810_3286_amd", "csrc", "svt_kernels.hip")


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


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


def cpu_baseline(p, seconds: float):
    """The oracle's one-sided Jacobi on a slab of the kick iterate, scaled.

    Algorithm 1 in the oracle takes a full Jacobi SVD of the dense m x n
    iterate each iteration: n(n-1)/2 column pairs per sweep.  The sample
    times the oracle on the first c columns of Y^{k0} (m x c, the same row
    length), growing c until the run takes about `seconds`; the per-pair cost
    and sweeps per SVD then give the oracle's time per SVT iteration at full
    size (sweeps per SVD taken from the sample itself).
    """
    import oracle.svt as osvt
    threads = 1  # the oracle's Jacobi is single-threaded C
    m, n = p.m, p.n
    # kick iterate columns: Y^{k0} = k0 delta P_Omega(M); k0 from the GPU-free
    # definition needs sigma_1 of P_Omega M, which is not needed for timing:
    # the Jacobi cost does not depend on the scale, so take P_Omega(M) itself.
    order = np.argsort(p.cols, kind="stable")
    cols_sorted = p.cols[order]
    c = 16
    elapsed = 0.0
    sweeps = 0
    while True:
        hi = np.searchsorted(cols_sorted, c)
        sel = order[:hi]
        A = np.zeros((m, c), order="F")
        A[p.rows[sel], p.cols[sel]] = p.vals[sel]
        V = np.zeros((c, c), order="F")
        s = np.zeros(c)
        t0 = time.perf_counter()
        sw = osvt._load().oracle_jacobi_svd(m, c, osvt._ptr(A), osvt._ptr(V), osvt._ptr(s),
                                            osvt.JACOBI_TOL, osvt.JACOBI_MAX_SWEEPS)
        elapsed = time.perf_counter() - t0
        sweeps = max(sw, 1)
        if elapsed >= seconds / 4 or c >= n:
            break
        c = min(n, c * 2)
    pairs_sample = c * (c - 1) / 2 * sweeps
    per_pair = elapsed / pairs_sample
    per_iter = per_pair * (n * (n - 1) / 2) * sweeps
    iters_per_s = 1.0 / per_iter
    return {
        "value": iters_per_s,
        "unit": "SVT iters/s",
        "sampled_entries_per_s": iters_per_s * p.nnz,
        "cores": threads,
        "kind": "oracle",
        "sample": (f"one-sided Jacobi (the oracle's full SVD) on a {m} x {c} column slab of "
                   f"P_Omega(M): {elapsed:.2f} s, {sweeps} sweeps; scaled by column pairs to the "
                   f"{m} x {n} iterate, {sweeps} sweeps per SVT iteration"),
    }


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
                  load_frac: float = 0.7, mix: str = "baseline", step_cap: int = 256):
    """Serving form on a stream of mixed completion requests.

    mix "baseline": m, n uniform in [500, 8000] (rectangular), r in
    {5, 10, 20, 50}, |Omega| = c r (m + n - r) with c uniform in [3, 6].
    mix "table1": m, n uniform in [1000, 8000] (aspect ratio at most 1.5),
    (r, c) drawn from Table 1's pairs (10, 6), (50, 5), (100, 4).
    Both: tau = 5 sqrt(m n), delta = 1.2 m n / |Omega|, eps = 1e-4, maxiter
    500, noise off; each request's bidiagonalisation is capped at step_cap
    steps (a request that needs more ends with SVT_ELANCZOS), so a request
    outside the method's regime holds its slot for a bounded time.
    Closed loop (all requests at t = 0) gives the capacity C in solves/s; an
    open loop with Poisson arrivals at load_frac * C gives the latency
    (arrival to completion) percentiles."""
    import threading
    import workload
    from paper_0810_3286_amd import svt as B
    if mix == "table1":
        trace = workload.serving_trace(2 * n_req, seed=seed, rate=1.0, mn_range=(1000, 8000),
                                       pairs=workload.TABLE1_RANK_OVERSAMPLING, max_aspect=1.5)
    else:
        trace = workload.serving_trace(2 * n_req, seed=seed, rate=1.0)
    probs = []
    for _, sp in trace:
        probs.append(workload.gaussian_lowrank(sp["m"], sp["n"], sp["r"], sp["nnz"], sp["seed"],
                                               noise_sigma=sp["noise_sigma"], maxiter=500))
        log(f"[bench] serving request {len(probs) - 1} generated ({sp['m']} x {sp['n']}, r {sp['r']}, "
            f"|Omega| {sp['nnz']})")

    def params(p):
        prm = B.svt_params_default(p.m, p.n, p.nnz)
        prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, p.delta, p.eps, p.maxiter, p.incr
        prm.precision = precision
        prm.lanczos_maxsteps = step_cap
        return prm

    budget = int(budget_gib * (1 << 30))
    srv = B.svt_server_create(budget, slots)
    statuses = []
    try:
        closed = probs[:n_req]
        t0 = time.perf_counter()
        tickets = [B.svt_submit(srv, p.m, p.n, p.rows, p.cols, p.vals, params(p)) for p in closed]
        iters = 0
        for i, t in enumerate(tickets):
            st, info = B.svt_wait(srv, t)
            iters += info.iters
            statuses.append(st)
            B.svt_release(srv, t)
            log(f"[bench] serving closed loop: request {i} done (status {st}, {info.iters} iterations)")
        t_closed = time.perf_counter() - t0
        capacity = n_req / t_closed
        log(f"[bench] serving closed loop: {n_req} solves in {t_closed:.2f} s")
        # open loop: Poisson arrivals at load_frac * capacity
        rate = load_frac * capacity
        rng = np.random.default_rng(seed + 1)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
        openp = probs[n_req:2 * n_req]
        tix = [None] * n_req

        def submitter():
            base = time.perf_counter()
            for i, p in enumerate(openp):
                dt = arrivals[i] - (time.perf_counter() - base)
                if dt > 0:
                    time.sleep(dt)
                tix[i] = B.svt_submit(srv, p.m, p.n, p.rows, p.cols, p.vals, params(p))
                log(f"[bench] serving open loop: request {i} submitted")

        t1 = time.perf_counter()
        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        lat = []
        for i, p in enumerate(openp):
            st, info = B.svt_wait(srv, tix[i])
            _, _, _, _, times = B.svt_result(srv, tix[i], p.m, p.n)
            lat.append(times[2] - times[0])
            statuses.append(st)
            B.svt_release(srv, tix[i])
            log(f"[bench] serving open loop: request {i} done (status {st}, latency {lat[-1]:.2f} s)")
        t_open = time.perf_counter() - t1
        stats = B.svt_server_stats(srv)
    finally:
        B.svt_server_destroy(srv)
    lat = np.array(lat)
    return {
        "requests_per_run": n_req, "slots": slots, "budget_gib": budget_gib,
        "precision": "mixed" if precision == B.SVT_MIXED else "fp64",
        "closed_loop_solves_per_s": capacity,
        "closed_loop_svt_iters_per_s": iters / t_closed,
        "mix": mix, "step_cap": step_cap,
        "status_counts": {B.svt_status_string(k): int(v) for k, v in
                          zip(*np.unique(np.array(statuses), return_counts=True))},
        "open_loop_rate_per_s": rate, "open_loop_solves_per_s": n_req / t_open,
        "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
        "max_running": stats["max_running"], "peak_admitted_gib": stats["peak_bytes"] / (1 << 30),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--profile-steps", type=int, default=1)
    ap.add_argument("--spmv-mode", type=int, default=0,
                    help="0: x in LDS when it fits in one segment, 1: gathered, 2: LDS segments")
    ap.add_argument("--serving-requests", type=int, default=16)
    ap.add_argument("--serving-slots", type=int, default=8)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-mix", choices=["baseline", "table1"], default="baseline")
    ap.add_argument("--serving-step-cap", type=int, default=256)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
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

    def make(profile):
        prm = B.svt_params_default(p.m, p.n, p.nnz)
        prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, p.delta, p.eps, p.maxiter, p.incr
        prm.precision = prec
        prm.profile = 1 if profile else 0
        prm.spmv_mode = args.spmv_mode
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
        "kernels": {KIND_NAMES[k]: {"launches": v[0], "ms": v[1],
                                    "avg_us": v[1] * 1e3 / max(v[0], 1),
                                    "GBps": (v[2] / (v[1] / 1e3) / 1e9) if v[1] > 0 else 0.0}
                    for k, v in kstats.items()},
        "roofline": {"kernel": KIND_NAMES[dom], "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": avg_s * 1e6},
    }
    if not args.no_fp64 and args.precision == "mixed":
        # the plain FP64 GPU solver on the same workload, for comparison
        prm = B.svt_params_default(p.m, p.n, p.nnz)
        prm.tau, prm.delta, prm.eps, prm.maxiter, prm.incr = p.tau, p.delta, p.eps, p.maxiter, p.incr
        prm.precision = B.SVT_FP64
        prm.spmv_mode = args.spmv_mode
        h64 = B.svt_create(p.m, p.n, p.rows, p.cols, p.vals, prm)
        try:
            log("[bench] fp64 comparison solves")
            B.svt_solve(h64)
            t0 = time.perf_counter()
            it64 = 0
            for _ in range(args.steps):
                _, inf = B.svt_solve(h64)
                it64 += inf.iters
            t64 = time.perf_counter() - t0
            U64, _, V64 = B.svt_factors(h64, p.m, p.n)
        finally:
            B.svt_destroy(h64)
        out["fp64"] = {"svt_iters_per_s": it64 / t64, "sampled_entries_per_s": it64 / t64 * p.nnz,
                       "iters_per_solve": it64 / args.steps, "ms_per_step": t64 / args.steps * 1e3,
                       "rel_error_vs_truth": rel_diff_factored(U64, V64, p.ML, p.MR),
                       "mixed_vs_fp64_rel_diff": rel_diff_factored(U, V, U64, V64)}
    if not args.no_serving:
        log("[bench] serving stream")
        out["serving"] = serving_bench(args.serving_requests, args.serving_slots, 64.0,
                                       B.SVT_MIXED if args.precision == "mixed" else B.SVT_FP64,
                                       mix=args.serving_mix, step_cap=args.serving_step_cap)
        out["solves_per_s"] = out["serving"]["closed_loop_solves_per_s"]
        out["p99_latency_s"] = out["serving"]["p99_latency_s"]
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
