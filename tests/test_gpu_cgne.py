"""CGNE through the C ABI against the oracle's CG and the dense solve.

Every solve must reach the FP64 true relative residual 1e-10 of D^+ D psi = eta. The
solution is compared with the oracle's solution: both satisfy |eta - A psi| <= 1e-10|eta|,
so they differ by at most 2e-10 * cond(A) relatively; cond(A) of these operators is
estimated from the dense 4^4 matrix (about 1e2), and the bound used is 1e-7.
"""
import numpy as np
import pytest

import oracle
from paper_2202_07388_amd import qdw
from paper_2202_07388_amd import synthetic as syn
from gpu_util import make_pair, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    dims = (4, 4, 4, 4)
    gop, oop, _, _ = make_pair(dims, 0.1, 1.5, 0.3, seed=7388)
    eta = syn.gaussian_spinor(dims, 7388 + 1000)
    return dims, gop, oop, eta


@pytest.fixture(scope="module")
def mid():
    dims = (16, 8, 8, 8)
    gop, oop, _, _ = make_pair(dims, -0.05, 1.7, 0.3, seed=7390)
    eta = syn.gaussian_spinor(dims, 7390 + 1000)
    xo, st = oracle.cgne(oop, eta, 1e-11, 5000)
    assert st > 0
    return dims, gop, oop, eta, xo


def _solve(gop, eta, **kw):
    e = gop.pack(eta, "f64")
    psi = gop.new_field("f64")
    info = qdw.cgne_solve(gop, e, psi, **kw)
    return gop.unpack(psi, "f64").cpu().numpy(), info


def test_cgne_fp64_small_matches_dense(small):
    dims, gop, oop, eta = small
    x, info = _solve(gop, eta, res=1e-10, inner="f64")
    assert info["status"] > 0 and info["rel_res_true"] <= 1e-10
    r = eta - oop.normal(x)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(eta)
    xo, st = oracle.cgne(oop, eta, 1e-10, 1000)
    assert rel(x, xo) <= 1e-7
    # FP64 CG with these settings only checks the true residual at the end (Sec. 2: the
    # binary64 curve never triggered a reset)
    assert info["nreset"] <= 1
    assert abs(info["status"] - st) <= 2


@pytest.mark.parametrize("inner", ["f64", "f32", "f16", "bf16"])
def test_cgne_precisions_reach_fp64_residual(mid, inner):
    dims, gop, oop, eta, xo = mid
    x, info = _solve(gop, eta, res=1e-10, inner=inner)
    assert info["status"] > 0, info
    assert info["rel_res_true"] <= 1e-10
    r = eta - oop.normal(x)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(eta)
    assert rel(x, xo) <= 1e-7
    if inner != "f64":
        assert info["nreset"] >= 1 and info["n_dw_lo"] == 2 * info["n_steps"]


def test_reset_count_grows_as_precision_drops(mid):
    """Sec. 2: with the paper's reset (restart after a drop of about the working epsilon)
    lower precision needs more reset steps: binary32 < binary16 < bfloat16."""
    dims, gop, oop, eta, xo = mid
    n = {}
    for inner in ("f32", "f16", "bf16"):
        x, info = _solve(gop, eta, res=1e-10, inner=inner, keep_p=False)
        assert info["status"] > 0 and info["rel_res_true"] <= 1e-10
        assert rel(x, xo) <= 1e-7
        n[inner] = info["nreset"]
    assert n["f32"] < n["f16"] < n["bf16"], n


def test_reliable_update_needs_fewer_steps_than_restart(mid):
    dims, gop, oop, eta, xo = mid
    _, keep = _solve(gop, eta, res=1e-10, inner="f32", keep_p=True)
    _, rest = _solve(gop, eta, res=1e-10, inner="f32", keep_p=False)
    _, plain = _solve(gop, eta, res=1e-10, inner="f64")
    assert keep["status"] > 0 and rest["status"] > 0
    assert keep["n_steps"] <= rest["n_steps"]
    # keeping the direction costs at most a few per cent more steps than FP64 CG
    assert keep["n_steps"] <= 1.1 * plain["n_steps"] + 5


def test_nmx_exhausted(mid):
    dims, gop, oop, eta, xo = mid
    _, info = _solve(gop, eta, res=1e-10, nmx=3)
    assert info["status"] == -1 and info["n_steps"] == 3
    assert 1e-10 < info["rel_res_true"] < 1


def test_fp16_without_resets_stagnates(mid):
    """Sec. 2: binary16 alone cannot get below ~1e-5; the solver must report stagnation
    (status -2) instead of running to nmx."""
    dims, gop, oop, eta, xo = mid
    _, info = _solve(gop, eta, res=1e-10, inner="f16", delta=0.0, nmx=5000)
    assert info["status"] == -2, info
    assert info["n_steps"] < 5000
    assert info["rel_res_true"] > 1e-10


def test_zero_source(small):
    dims, gop, oop, eta = small
    x, info = _solve(gop, np.zeros_like(eta), res=1e-10)
    assert info["status"] == 0 and np.abs(x).max() == 0


# ---------------------------------------------------------------- precision cascade

@pytest.mark.parametrize("c", [1.0, 10.0])
def test_cascade_reaches_fp64_residual(mid, c):
    """BF16 -> FP32 -> FP64 (Sec. 2.1): the FP64 true residual 1e-10 is reached, the
    solution agrees with the oracle's, and the FP64 phase takes only the last few digits:
    far fewer FP64 operator applications than plain FP64 CG."""
    dims, gop, oop, eta, xo = mid
    x, info = _solve(gop, eta, res=1e-10, cascade=True, cascade_c=c)
    assert info["status"] > 0 and info["rel_res_true"] <= 1e-10, info
    r = eta - oop.normal(x)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(eta)
    assert rel(x, xo) <= 1e-7
    _, plain = _solve(gop, eta, res=1e-10, inner="f64")
    # all of plain FP64 CG's applications are FP64 (its regular steps count as n_dw_lo)
    assert info["n_dw_lo"] > 0 and info["n_dw_hi"] < 0.5 * (plain["n_dw_hi"] + plain["n_dw_lo"])


def test_cascade_phases_follow_the_thresholds(mid):
    """A target above the BF16 switch point is met by the BF16 phase alone (no FP64
    operator applications beyond the residual checks); one between the switch points
    needs BF16 and FP32 only."""
    dims, gop, oop, eta, xo = mid
    _, a = _solve(gop, eta, res=2e-2, cascade=True, cascade_c=1.0)
    assert a["status"] > 0 and a["rel_res_true"] <= 2e-2
    # FP64 applications: 2 per reset of the BF16 phase, 2 for its final check and 2 for
    # the cascade's residual after the phase (counted as one more reset)
    assert a["n_dw_hi"] == 2 * a["nreset"] + 2
    _, b = _solve(gop, eta, res=1e-5, cascade=True, cascade_c=1.0)
    assert b["status"] > 0 and b["rel_res_true"] <= 1e-5
    assert b["n_steps"] > a["n_steps"]


def test_cascade_zero_source(mid):
    dims, gop, oop, eta, xo = mid
    x, info = _solve(gop, np.zeros_like(eta), res=1e-10, cascade=True)
    assert info["status"] == 0 and np.abs(x).max() == 0.0
