"""Solves and the network at the benchmark's full sizes, in the configurations it times (the
D-kernel shapes pinned as in bench.py), through the C ABI.

The oracle cannot solve at these sizes, so the checks are properties that hold at any
size: every solve must reach the FP64 true residual 1e-10, recomputed here independently
with the library's FP64 operators (which test_gpu_dirac pins against the oracle on sampled
sites at 32^3 x 64, in these shapes), and with identity weights the network must return
its input exactly. The network with random weights, in the benchmark's bf16 mixing and in
FP32 mixing, is compared with the oracle on sampled sites (oracle.nn_at_sites).
"""
import numpy as np
import pytest

import oracle
from paper_2202_07388_amd import qdw
from paper_2202_07388_amd import synthetic as syn

pytestmark = pytest.mark.gpu


def _norm(t):
    import torch
    return float(torch.linalg.vector_norm(t))


def _even_mask(dims, device):
    import torch
    T, L1, L2, L3 = dims
    x0, x1, x2, x3 = np.meshgrid(np.arange(T), np.arange(L1), np.arange(L2), np.arange(L3),
                                 indexing="ij")
    even = ((x0 + x1 + x2 + x3) % 2 == 0).reshape(-1)
    return torch.as_tensor(even, device=device)


@pytest.fixture(scope="module")
def op32(gauge32):
    from bench import CSW, DIMS, M0, PINNED_SHAPES, SEED
    su3, th = gauge32
    op = qdw.Op(DIMS, su3, th, M0, CSW, -1)
    for p, shape in PINNED_SHAPES.items():
        qdw.set_dw_shape(op, p, *shape)
    eta = op.pack(syn.gaussian_spinor(DIMS, SEED + 1000))
    yield DIMS, op, eta
    op.close()


@pytest.mark.parametrize("kw", [dict(inner="f16"), dict(inner="f16", schur=True)])
def test_cgne_full_size(op32, kw):
    """D^+ D psi = eta (or the even-odd reduced D^+ D^ psi_e = eta_e) at 32^3 x 64 with FP16
    regular steps and FP64 reset steps, the benchmark's chosen forms."""
    dims, op, eta = op32
    psi = op.new_field()
    info = qdw.cgne_solve(op, eta, psi, res=1e-10, nmx=20000, **kw)
    assert info["status"] > 0 and info["rel_res_true"] <= 1e-10, info
    t, y = op.new_field(), op.new_field()
    if kw.get("schur"):
        qdw.dw_schur_apply(op, psi, t)
        qdw.dw_schur_dag_apply(op, t, y)
        even = _even_mask(dims, op.device)
        e = op.unpack(eta)[even]
        r = e - op.unpack(y)[even]
        assert _norm(op.unpack(psi)[~even]) == 0.0  # the odd half stays zero
    else:
        qdw.dw_apply(op, psi, t)
        qdw.dw_dag_apply(op, t, y)
        e = op.unpack(eta)
        r = e - op.unpack(y)
    assert _norm(r) <= 1.01e-10 * _norm(e), (_norm(r) / _norm(e), info)


@pytest.fixture(scope="module")
def op24():
    from bench import CSW, EPS_U1, SAP_DIMS, SAP_EPS, SAP_M0, SAP_SEED
    su3, th = syn.gauge_field(SAP_DIMS, SAP_EPS, EPS_U1, SAP_SEED)
    op = qdw.Op(SAP_DIMS, su3, th, SAP_M0, CSW, -1)
    del su3, th
    eta = op.pack(syn.gaussian_spinor(SAP_DIMS, SAP_SEED + 1000))
    yield op, eta
    op.close()


@pytest.mark.parametrize("precond", ["sap", "sap_eo"])
def test_sap_gcr_full_size(op24, precond):
    """D psi = eta at 24^3 x 48 with FP16 SAP on 4^4 blocks (5 cycles, 4 MR steps), plain or
    with even-odd reduced block solves, as the benchmark runs it."""
    op, eta = op24
    psi = op.new_field()
    info = qdw.sap_gcr_solve(op, eta, psi, res=1e-10, nmx=5000, nkv=16, ncy=5, nmr=4,
                             bs=(4, 4, 4, 4), sdtype="f16", precond=precond)
    assert info["status"] > 0 and info["rel_res_true"] <= 1e-10, info
    assert info["status"] < 30, info  # plain GCR needs 124 steps here
    t = op.new_field()
    qdw.dw_apply(op, psi, t)
    e = op.unpack(eta)
    r = e - op.unpack(t)
    assert _norm(r) <= 1.01e-10 * _norm(e), (_norm(r) / _norm(e), info)


def test_network_identity_full_size(op32):
    """Identity weights (the identity path with weight 1, every other weight 0) return the
    input exactly at 32^3 x 64 (FP32 matrix-core mixing)."""
    import torch
    dims, op, eta = op32
    w = qdw.nn_weights_tensor(oracle.nn_identity_weights())
    src = syn.gaussian_spinor(dims, 4321)
    x = op.pack(src)
    y = op.new_field()
    qdw.nn_forward(op, w, x, y, f32_mixing=True)
    got = op.unpack(y)
    want = torch.as_tensor(src.real.astype(np.float32).astype(np.float64)
                           + 1j * src.imag.astype(np.float32).astype(np.float64),
                           device=op.device)
    assert torch.equal(got, want)


@pytest.mark.parametrize("f32,tol", [(False, 1e-2), (True, 1e-5)])
def test_network_random_weights_sampled_sites(op32, gauge32, f32, tol):
    """The network at 32^3 x 64 with random (non-identity) weights, as the benchmark
    evaluates it (bf16 operands on the matrix cores, FP32 accumulation) and with FP32
    mixing, against the oracle on 256 sampled sites including the time boundary and the
    lattice corners. Tolerances as in test_gpu_nn (bf16 rounding u = 2^-9 of the operands)."""
    dims, op, _ = op32
    su3, th = gauge32
    u = oracle.u3_links(su3, th)
    W = oracle.nn_identity_weights(seed=5, scale=0.3)
    src = syn.gaussian_spinor(dims, 4322)
    rng = np.random.default_rng(7)
    V = int(np.prod(dims))
    x = np.array([[0, 0, 0, 0], [63, 31, 31, 31], [63, 0, 31, 0], [0, 31, 0, 31]])
    lex = list(((x[:, 0] * 32 + x[:, 1]) * 32 + x[:, 2]) * 32 + x[:, 3])
    sites = np.array(lex + list(rng.integers(0, V, 252)))
    want = oracle.nn_at_sites(dims, -1, u, W, src, sites)
    y = op.new_field()
    qdw.nn_forward(op, qdw.nn_weights_tensor(W), op.pack(src), y, f32_mixing=f32)
    got = op.unpack(y)[sites].cpu().numpy()
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err <= tol, err
