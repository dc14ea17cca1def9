"""Parity of the HIP Wilson-clover operator with the FP64 oracle.

Tolerances: FP64 1e-13 (relative, norm and max) as the operator is a fixed short sum
of products; FP32 2e-6 (relative norm); FP16 / BF16 storage with FP32 arithmetic: every
input (spinor, link rows, phase, clover) and the output are rounded once to the storage
format (unit roundoff u = 2^-11 for FP16, 2^-8 for BF16), and the output is a sum of
nine terms of comparable size, so the relative error is a few u: 4u is required.
"""
import numpy as np
import pytest

import oracle
from paper_2202_07388_amd import qdw
from paper_2202_07388_amd import synthetic as syn
from gpu_util import make_pair, rel, maxrel

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 2e-6, "f16": 4 * 2.0 ** -11, "bf16": 4 * 2.0 ** -8}

CASES = [
    # (dims, m0, csw, eps, bc)
    ((4, 4, 4, 4), 0.1, 1.5, 0.3, -1),       # the 4^4 correctness workload
    ((16, 8, 8, 8), -0.05, 1.7, 0.3, -1),    # 8^3 x 16, 32 workgroups
    ((6, 4, 4, 6), -0.05, 1.7, 0.35, -1),    # V/2 = 288: ragged last workgroup
    ((10, 6, 6, 12), 0.2, 1.0, 0.3, +1),     # ragged, periodic time
    ((2, 2, 2, 2), 0.0, 1.0, 0.5, -1),       # smallest lattice: x+mu and x-mu coincide
]


@pytest.fixture(scope="module", params=range(len(CASES)))
def case(request):
    dims, m0, csw, eps, bc = CASES[request.param]
    gop, oop, su3, th = make_pair(dims, m0, csw, eps, seed=100 + request.param, bc=bc)
    psi = syn.gaussian_spinor(dims, 500 + request.param)
    return dims, gop, oop, psi


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("dag", [False, True])
def test_dw_parity(case, prec, dag):
    dims, gop, oop, psi = case
    x = gop.pack(psi, prec)
    y = gop.new_field(prec)
    (qdw.dw_dag_apply if dag else qdw.dw_apply)(gop, x, y, prec)
    got = gop.unpack(y, prec).cpu().numpy()
    want = (oop.dw_dag if dag else oop.dw)(psi)
    assert rel(got, want) <= TOL[prec], (dims, prec, dag, rel(got, want))
    if prec == "f64":
        assert maxrel(got, want) <= 1e-13


@pytest.mark.parametrize("dag", [False, True])
def test_full_links_control(case, dag):
    """The uncompressed control (links read as full 3x3 matrices) against the oracle at the
    FP64 bar, and against the compressed kernel: the third rows are formed by the same
    FP64 expression, so only the order of the final sums can differ (a few ulp)."""
    dims, gop, oop, psi = case
    x = gop.pack(psi, "f64")
    qdw.set_full_links(gop)
    got = gop.new_field("f64")
    qdw.dw_apply_full_links(gop, x, got, dagger=dag)
    ref = gop.new_field("f64")
    (qdw.dw_dag_apply if dag else qdw.dw_apply)(gop, x, ref, "f64")
    g = gop.unpack(got, "f64").cpu().numpy()
    want = (oop.dw_dag if dag else oop.dw)(psi)
    assert rel(g, want) <= TOL["f64"] and maxrel(g, want) <= TOL["f64"]
    assert maxrel(g, gop.unpack(ref, "f64").cpu().numpy()) <= 1e-14


def test_full_links_need_setting_first():
    dims = (4, 4, 4, 4)
    su3, th = syn.gauge_field(dims, 0.3, 0.1, 17)
    gop = qdw.Op(dims, su3, th, 0.1, 1.5, -1)
    x = gop.pack(syn.gaussian_spinor(dims, 18), "f64")
    with pytest.raises(qdw.QdwError, match="full links"):
        qdw.dw_apply_full_links(gop, x, gop.new_field("f64"))


def test_pack_unpack_round_trip():
    dims = (6, 4, 4, 6)
    su3, th = syn.gauge_field(dims, 0.3, 0.1, 3)
    gop = qdw.Op(dims, su3, th, 0.1, 1.5)
    psi = syn.gaussian_spinor(dims, 4)
    for prec in ("f64", "f32", "f16", "bf16"):
        back = gop.unpack(gop.pack(psi, prec), prec).cpu().numpy()
        if prec == "f64":
            assert np.array_equal(back, psi)
        else:
            dt = {"f32": np.float32, "f16": np.float16}.get(prec)
            if dt is not None:
                want = psi.real.astype(dt).astype(np.float64) + 1j * psi.imag.astype(dt).astype(np.float64)
                assert np.array_equal(back, want), prec
            else:
                assert rel(back, psi) <= 2.0 ** -8


def test_fp16_format_limits_from_table():
    """Values at the binary16 limits of the paper's Table 1 survive FP16 storage exactly."""
    dims = (2, 2, 2, 2)
    su3, th = syn.unit_gauge_field(dims)
    gop = qdw.Op(dims, su3, th, 0.0, 0.0)
    psi = np.zeros((16, 4, 3), dtype=np.complex128)
    psi[0, 0, 0] = 65504.0             # f_max
    psi[1, 0, 0] = 2.0 ** -14          # f_min (smallest normal)
    psi[2, 0, 0] = 2.0 ** -24          # f_smin (smallest subnormal)
    psi[3, 0, 0] = 1.0 + 2.0 ** -10    # 1 + eps
    back = gop.unpack(gop.pack(psi, "f16"), "f16").cpu().numpy()
    assert np.array_equal(back, psi)


def test_dw_deterministic():
    dims = (16, 8, 8, 8)
    gop, oop, _, _ = make_pair(dims, -0.05, 1.7, seed=9)
    x = gop.pack(syn.gaussian_spinor(dims, 10), "f64")
    a, b = gop.new_field("f64"), gop.new_field("f64")
    qdw.dw_apply(gop, x, a, "f64")
    qdw.dw_apply(gop, x, b, "f64")
    import torch
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_rejects_non_unitary_links():
    dims = (2, 2, 2, 2)
    su3, th = syn.unit_gauge_field(dims)
    su3[3, 1, 0, 0] = 1.001
    with pytest.raises(qdw.QdwError, match="SU\\(3\\)"):
        qdw.Op(dims, su3, th, 0.0, 1.0)


def test_rejects_odd_extent():
    dims = (4, 4, 4, 3)
    su3, th = syn.unit_gauge_field(dims)
    with pytest.raises(qdw.QdwError, match="even"):
        qdw.Op(dims, su3, th, 0.0, 1.0)


def test_full_size_sampled_sites(gauge32):
    """32^3 x 64 in the launch configurations the benchmark times (its pinned shapes) and
    in the one-workgroup-per-slice form, D and D^+, checked on sampled sites that the
    oracle computes one by one (FP64 to 1e-13, FP32 to 2e-6, FP16 storage to 2e-2)."""
    dims = (64, 32, 32, 32)
    su3, th = gauge32  # eps 0.3, U(1) 0.1, seed 7388 + 10
    m0, csw = -0.05, 1.7
    gop = qdw.Op(dims, su3, th, m0, csw)
    psi = syn.gaussian_spinor(dims, 7388 + 10 + 1000)
    u = oracle.u3_links(su3, th)
    rng = np.random.default_rng(1)
    V = int(np.prod(dims))
    # corners and faces (wrap-around, time boundary) plus random interior sites
    x = np.array([[0, 0, 0, 0], [63, 31, 31, 31], [63, 0, 31, 0], [0, 31, 0, 31],
                  [31, 15, 0, 31]])
    lex = list(((x[:, 0] * 32 + x[:, 1]) * 32 + x[:, 2]) * 32 + x[:, 3])
    sites = np.array(lex + list(rng.integers(0, V, 251)))
    want = oracle.dw_at_sites(dims, -1, u, m0, csw, psi, sites)
    # D^+ = gamma_5 D gamma_5 (pinned in the oracle tests), sampled the same way
    g5 = np.array([1.0, 1.0, -1.0, -1.0])[None, :, None]
    want_dag = g5 * oracle.dw_at_sites(dims, -1, u, m0, csw, g5[0] * psi, sites)
    from bench import PINNED_SHAPES  # the shapes the benchmark times
    for prec, tol in (("f64", 1e-13), ("f32", 2e-6), ("f16", 2e-2)):
        xf = gop.pack(psi, prec)
        for shape in (PINNED_SHAPES[prec], None):
            if shape is not None:
                qdw.set_dw_shape(gop, prec, *shape)
            else:
                qdw.set_dw_shape(gop, prec, 128, 8, 1, 0, 0)  # the one-workgroup-per-slice form
            for dag in (False, True):
                y = gop.new_field(prec)
                (qdw.dw_dag_apply if dag else qdw.dw_apply)(gop, xf, y, prec)
                got = gop.unpack(y, prec)[sites].cpu().numpy()
                ref = want_dag if dag else want
                assert rel(got, ref) <= tol, (prec, shape, dag, rel(got, ref))
