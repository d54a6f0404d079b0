"""Reorthogonalisation modes on the GPU (needs an MI355X).

The bidiagonalisation orthogonalises each new vector against the whole basis
by classical Gram-Schmidt: one pass by default (restarting with two passes
when a pass removes more than half of a vector's |.|^2, the DGKS criterion),
always one, or always two.  All three reach the oracle's result; the default
equals the one-pass mode bit for bit when the check never fires, and a
forced restart (threshold 0) still reaches the two-pass result."""
import os

import numpy as np
import pytest

import workload
from paper_0810_3286_amd import solve
from paper_0810_3286_amd import svt as B
from tests.helpers import gpu_case, rel_diff_factored

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _solve(p, **kw):
    return solve(p.m, p.n, p.rows, p.cols, p.vals, tau=p.tau, delta=p.delta, eps=p.eps,
                 maxiter=p.maxiter, incr=p.incr, **kw)


@pytest.mark.parametrize("passes", [0, 1, 2])
def test_modes_match_stored_oracle_400(passes):
    gpu_case(f"400^2 FP64 reorth_passes {passes} vs stored oracle")
    p = workload.config(1)
    o = np.load(os.path.join(GOLDEN, "oracle_config1.npz"))
    g = _solve(p, reorth_passes=passes)
    assert g["status"] == B.SVT_OK and g["info"]["iters"] == int(o["iters"])
    assert list(g["ranks"]) == list(o["ranks"])
    np.testing.assert_allclose(g["residuals"], o["residuals"], rtol=1e-8)
    assert rel_diff_factored(g["U"], g["V"], o["U"], o["V"]) <= 1e-8


@pytest.mark.parametrize("precision", [B.SVT_FP64, B.SVT_MIXED])
def test_default_equals_one_pass(precision):
    gpu_case(f"reorth default vs one pass, precision {precision}")
    p = workload.gaussian_lowrank(300, 260, 6, 30000, 12, maxiter=300)
    a = _solve(p, precision=precision, reorth_passes=0)
    b = _solve(p, precision=precision, reorth_passes=1)
    assert a["info"]["iters"] == b["info"]["iters"] and list(a["ranks"]) == list(b["ranks"])
    assert np.array_equal(a["U"], b["U"]) and np.array_equal(a["V"], b["V"])


def test_forced_restart_reaches_two_pass_result(capfd, monkeypatch):
    gpu_case("reorth restart forced by a zero threshold")
    p = workload.gaussian_lowrank(300, 260, 6, 30000, 12, maxiter=300)
    two = _solve(p, reorth_passes=2)
    monkeypatch.setenv("SVT_REORTH_TRIGGER", "0")
    monkeypatch.setenv("SVT_LOG", "1")
    forced = _solve(p, reorth_passes=0)
    err = capfd.readouterr().err
    assert "restarting with two passes" in err
    assert forced["info"]["iters"] == two["info"]["iters"]
    assert list(forced["ranks"]) == list(two["ranks"])
    # the restart draws a new start vector: the same triplets to rounding
    assert rel_diff_factored(forced["U"], forced["V"], two["U"], two["V"]) <= 1e-9
