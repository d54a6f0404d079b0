"""Partial reorthogonalisation of the bidiagonalisation (Section 5.1.1;
svt_params.reorth_eta) on the GPU, against the oracle.

With reorth_eta > 0 a new vector of the bidiagonalisation is orthogonalised
against its basis only when the estimate of its loss of orthogonality is
predicted to pass reorth_eta sqrt(u) (u the unit roundoff of the vectors);
the bases stay semi-orthogonal and the Ritz
triplets, hence every SVT iterate, agree with the oracle's to the same
tolerances as with full reorthogonalisation:

* the small solves of ``test_gpu_parity`` against tier A and the 400^2
  stored run: same iterations, ranks and s_k, X within 1e-8;
* the stored oracle runs at full size: 5000^2 X^60, 10000^2 rank 50 X^40
  and its complete run, 30000^2 X^20 and its complete run: FP64 within 1e-8
  with the same ranks, while fewer than a quarter of the vectors are
  orthogonalised (a third over the first 20 iterations at 30000^2, whose
  first bidiagonalisations have no previous pattern to follow) and none
  falls back; the mixed form (FP32 vectors, the automatic level 0.1)
  within 5e-4 while orthogonalising fewer vectors than with reorth_eta = 0;
  the automatic level is 0.01 (FP64) and 0.1 (FP32) bit for bit;
* the fall-back: reorth_eta = 100 lets predictions pass sqrt(u), the check
  of the estimates must then restart with full reorthogonalisation, and the
  solve still matches the oracle;
* with two Gram-Schmidt passes (reorth_passes = 2) partial
  reorthogonalisation stays off.
"""
import os

import numpy as np
import pytest

import oracle
import workload
from paper_0810_3286_amd import solve
from paper_0810_3286_amd import svt as B
from tests.helpers import gpu_case, rel_diff_factored
from tests.test_gpu_fullsize import GOLDEN, _gold
from tests.test_gpu_parity import SOLVE_CASES, _compare_solves

pytestmark = pytest.mark.gpu

ETA = 0.01


def _run(p, precision=B.SVT_FP64, eta=ETA, k=None, **kw):
    # eta None: the library's automatic level
    if eta is not None:
        kw["reorth_eta"] = eta
    return solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta,
                 eps=0.0 if k else p.eps, maxiter=k or p.maxiter, incr=p.incr,
                 precision=precision, **kw)


def _stats(g):
    vectors, orth, two_pass, fallbacks = g["reorth"]
    assert vectors > 0 and two_pass == 0
    return orth / vectors, fallbacks


@pytest.mark.parametrize("case", SOLVE_CASES)
def test_small_solves_match_tier_a(case):
    m, n, r, nnz, seed = case
    gpu_case(f"partial reorth: solve {case}")
    p = workload.gaussian_lowrank(m, n, r, nnz, seed, maxiter=300, shuffle=True)
    g = _run(p)
    o = oracle.svt_dense(p.m, p.n, p.rows, p.cols, p.vals, p.tau, p.delta, p.eps, p.maxiter, p.incr)
    _compare_solves(g, o)
    assert list(g["s_hist"]) == list(o["s_hist"])
    assert _stats(g)[1] == 0


def test_400_matches_stored_oracle():
    gpu_case("partial reorth: 400^2 vs stored oracle")
    p = workload.config(1)
    gold = np.load(os.path.join(GOLDEN, "oracle_config1.npz"))
    g = _run(p)
    o = dict(status="ok", k0=int(gold["k0"]), iters=int(gold["iters"]), ranks=list(gold["ranks"]),
             residuals=gold["residuals"], U=gold["U"], V=gold["V"])
    _compare_solves(g, o)
    assert list(g["s_hist"]) == list(gold["s_hist"])
    frac, fallbacks = _stats(g)
    assert fallbacks == 0 and frac < 0.25


@pytest.mark.parametrize("cfg,k,frac_max", [(2, 60, 0.25), (3, 40, 0.25), (4, 20, 0.33)])
def test_fixed_iteration_matches_stored_oracle(cfg, k, frac_max):
    gpu_case(f"partial reorth: config {cfg} FP64, {k} iterations vs stored oracle")
    p = workload.config(cfg)
    o = _gold(f"{cfg}_k{k}")
    g = _run(p, k=k)
    assert g["info"]["iters"] == k == o["iters"] and g["info"]["k0"] == o["k0"]
    assert list(g["ranks"]) == o["ranks"]
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=1e-8)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 1e-8
    frac, fallbacks = _stats(g)
    assert fallbacks == 0 and frac < frac_max


@pytest.mark.parametrize("cfg", [3, 4])
def test_complete_run_matches_stored_oracle(cfg):
    gpu_case(f"partial reorth: config {cfg} FP64 complete run vs stored oracle")
    p = workload.config(cfg)
    o = _gold(cfg)
    g = _run(p)
    assert g["status"] == B.SVT_OK
    assert g["info"]["iters"] == o["iters"] and g["info"]["k0"] == o["k0"]
    assert list(g["ranks"]) == o["ranks"]
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=1e-8)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 1e-8
    frac, fallbacks = _stats(g)
    assert fallbacks == 0 and frac < 0.25


@pytest.mark.parametrize("cfg,k", [(2, 60), (4, 20)])
def test_mixed_matches_stored_oracle(cfg, k):
    gpu_case(f"partial reorth: config {cfg} mixed, {k} iterations vs stored oracle")
    p = workload.config(cfg)
    o = _gold(f"{cfg}_k{k}")
    g = _run(p, precision=B.SVT_MIXED, eta=None, k=k)
    assert list(g["ranks"]) == o["ranks"]
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=5e-4)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 5e-4


def test_fallback_to_full_reorthogonalisation():
    gpu_case("partial reorth: FP64 with eta 100 falls back to full")
    p = workload.config(2)
    o = _gold("2_k60")
    g = _run(p, eta=100.0, k=60)
    frac, fallbacks = _stats(g)
    assert fallbacks >= 1          # each bidiagonalisation whose check fails
    assert list(g["ranks"]) == o["ranks"]
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=1e-8)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 1e-8


@pytest.mark.parametrize("cfg", [1, 3])
def test_mixed_default_orthogonalises_fewer(cfg):
    # FP32 vectors at the default level: fewer vectors orthogonalised than
    # with level 0, no fall-back, and the same result to the mixed bar
    gpu_case(f"partial reorth: config {cfg} mixed, default vs level 0")
    p = workload.config(cfg)
    k = 30
    a = _run(p, precision=B.SVT_MIXED, eta=None, k=k)
    b = _run(p, precision=B.SVT_MIXED, eta=0.0, k=k)
    fa, fall = _stats(a)
    fb, _ = _stats(b)
    assert fall == 0 and fa < 0.9 * fb
    assert list(a["ranks"]) == list(b["ranks"])
    assert rel_diff_factored(a["U"], a["V"], b["U"], b["V"]) <= 5e-4


@pytest.mark.parametrize("precision,level", [(B.SVT_FP64, 0.01), (B.SVT_MIXED, 0.1)])
def test_automatic_level(precision, level):
    # the default (negative) level: 0.01 sqrt(u) for FP64 vectors, 0.1 sqrt(u)
    # for FP32 vectors, bit for bit
    gpu_case(f"partial reorth: automatic level, precision {precision}")
    p = workload.config(1)
    a = _run(p, precision=precision, eta=None, k=40)
    b = _run(p, precision=precision, eta=level, k=40)
    np.testing.assert_array_equal(a["U"], b["U"])
    np.testing.assert_array_equal(a["V"], b["V"])
    assert a["reorth"] == b["reorth"]


def test_two_passes_keep_full_reorthogonalisation():
    gpu_case("partial reorth: reorth_passes 2 ignores eta")
    p = workload.config(1)
    g = _run(p, k=20, reorth_passes=2)
    frac, fallbacks = _stats(g)
    assert fallbacks == 0 and frac > 0.9
