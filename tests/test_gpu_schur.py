"""The even-odd reduced operator D^ = A_ee - D_eo A_oo^-1 D_oe and CGNE on its normal
equations, through the C ABI, against the oracle's definition from the blocks of D.

Bars: D^ in FP64 within 1e-13 relative (max-norm over the even half; A_oo^-1 is formed in
FP64 on both sides, by Gauss-Jordan on the GPU and by LAPACK in the oracle), FP32 within
2e-6; with FP16/BF16 storage every component within 1.25 times the first-order
rounding-error bound of schur_bound.py (each stored input, link row, determinant, clover
entry, inverse entry, intermediate and output rounded with the format's unit roundoff,
propagated entry by entry); solves reach the FP64 true residual 1e-10 of the reduced
normal equations (checked with the oracle) and agree with the oracle's solution to 1e-7.
"""
import numpy as np
import pytest

import oracle
from paper_2202_07388_amd import qdw
from paper_2202_07388_amd import synthetic as syn
from gpu_util import make_pair, maxrel, rel
from schur_bound import schur_error_bound

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 2e-6}
UNIT_ROUNDOFF = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}


@pytest.fixture(scope="module", params=[(4, 4, 4, 4), (6, 4, 6, 10), (8, 8, 8, 8)])
def lat(request):
    dims = request.param
    gop, oop, _, _ = make_pair(dims, -0.05, 1.7, 0.3, seed=61)
    return dims, gop, oop, oracle.Schur(oop)


def _even(sc, v):
    return np.asarray(v).reshape(-1, 4, 3)[sc.even[:, 0, 0]]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_schur_apply_matches_oracle(lat, prec):
    dims, gop, oop, sc = lat
    v = syn.gaussian_spinor(dims, 62)
    x = gop.pack(v, prec)
    out = gop.new_field(prec)
    for dag in (False, True):
        (qdw.dw_schur_dag_apply if dag else qdw.dw_schur_apply)(gop, x, out, prec)
        got = gop.unpack(out, prec).cpu().numpy()
        want = sc.apply_dag(v) if dag else sc.apply(v)
        if prec in TOL:
            assert maxrel(_even(sc, got), _even(sc, want)) <= TOL[prec]
        else:
            bound, _ = schur_error_bound(oop, sc, v, UNIT_ROUNDOFF[prec], dag=dag)
            err = np.abs(_even(sc, got) - _even(sc, want))
            assert np.all(err <= 1.25 * _even(sc, bound)), (prec, dag, float(
                (err / np.maximum(_even(sc, bound), 1e-300)).max()))


def test_schur_ignores_the_odd_half(lat):
    """Odd components of the input do not change the result."""
    import torch
    dims, gop, oop, sc = lat
    v = syn.gaussian_spinor(dims, 63)
    w = np.where(sc.even, v, syn.gaussian_spinor(dims, 64))
    a, b = gop.new_field(), gop.new_field()
    qdw.dw_schur_apply(gop, gop.pack(v), a)
    qdw.dw_schur_apply(gop, gop.pack(w), b)
    ga, gb = gop.unpack(a).cpu().numpy(), gop.unpack(b).cpu().numpy()
    assert np.array_equal(_even(sc, ga), _even(sc, gb))


@pytest.fixture(scope="module")
def mid():
    dims = (16, 8, 8, 8)
    gop, oop, _, _ = make_pair(dims, -0.05, 1.7, 0.3, seed=7390)
    sc = oracle.Schur(oop)
    eta = syn.gaussian_spinor(dims, 7390 + 1000)
    xo, st = oracle.cgne_schur(sc, eta, 1e-11, 5000)
    assert st > 0
    return dims, gop, oop, sc, eta, xo


def _solve(gop, eta, **kw):
    e = gop.pack(eta, "f64")
    psi = gop.new_field("f64")
    info = qdw.cgne_solve(gop, e, psi, **kw)
    return gop.unpack(psi, "f64").cpu().numpy(), info


@pytest.mark.parametrize("kw", [dict(inner="f64"), dict(inner="f32"), dict(inner="f16"),
                                dict(cascade=True)])
def test_cgne_schur_reaches_fp64_residual(mid, kw):
    dims, gop, oop, sc, eta, xo = mid
    x, info = _solve(gop, eta, res=1e-10, schur=True, **kw)
    assert info["status"] > 0 and info["rel_res_true"] <= 1e-10, info
    ee = np.where(sc.even, eta, 0)
    assert np.linalg.norm(ee - sc.normal(x)) <= 1.01e-10 * np.linalg.norm(ee)
    assert np.abs(np.where(sc.odd, x, 0)).max() == 0.0
    assert rel(_even(sc, x), _even(sc, xo)) <= 1e-7


def test_schur_cuts_the_iteration_count(mid):
    """The reduced system is better conditioned: fewer CG steps than the full normal
    equations for the same source and target."""
    dims, gop, oop, sc, eta, xo = mid
    _, red = _solve(gop, eta, res=1e-10, schur=True, inner="f64")
    _, full = _solve(gop, eta, res=1e-10, inner="f64")
    assert red["status"] > 0 and full["status"] > 0
    assert red["status"] < 0.7 * full["status"], (red, full)
