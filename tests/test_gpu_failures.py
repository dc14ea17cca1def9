"""Failure paths and memory ownership on the GPU.

A solve that meets a non-finite value reports status -3 and still returns a finite
iterate (the last finite one); the learned preconditioner hands a solve to SAP when its
output is not finite; and an operator's device memory is a torch allocation of exactly the
size the library asks for. The non-finite values come from the host side (an operator
whose mass overflows D^+ D, network weights set to NaN); every kernel runs to its end.
"""
import numpy as np
import pytest

from paper_2202_07388_amd import qdw
from paper_2202_07388_amd import synthetic as syn
from gpu_util import make_pair

pytestmark = pytest.mark.gpu

DIMS = (8, 4, 4, 8)


@pytest.fixture(scope="module")
def huge():
    """m0 = 1e200: D p is finite, |D p|^2 overflows to infinity in the first CG step."""
    su3, th = syn.gauge_field(DIMS, 0.3, 0.1, 61)
    return qdw.Op(DIMS, su3, th, 1e200, 1.5, -1)


@pytest.mark.parametrize("inner", ["f64", "f32", "f16"])
def test_cgne_non_finite_returns_a_finite_iterate(huge, inner):
    import torch
    eta = huge.pack(syn.gaussian_spinor(DIMS, 62), "f64")
    psi = huge.new_field("f64")
    info = qdw.cgne_solve(huge, eta, psi, res=1e-10, nmx=50, inner=inner)
    assert info["status"] == -3, info
    x = huge.unpack(psi, "f64")
    assert bool(torch.isfinite(x).all())
    assert np.isfinite(info["rel_res_true"])


def test_gcr_non_finite_returns_a_finite_iterate():
    """m0 = 1e308: D phi itself overflows to infinity in some components, the step's
    Gram-Schmidt turns them into NaN, the column is dropped and the solve ends with -3 and
    the iterate of the finite columns (here psi = 0). (A milder overflow, where only |D phi|
    is infinite, makes the step a no-op instead: 1/|chi| = 0.)"""
    import torch
    su3, th = syn.gauge_field(DIMS, 0.3, 0.1, 61)
    op = qdw.Op(DIMS, su3, th, 1e308, 1.5, -1)
    eta = op.pack(syn.gaussian_spinor(DIMS, 63), "f64")
    psi = op.new_field("f64")
    info = qdw.sap_gcr_solve(op, eta, psi, res=1e-10, nmx=50, nkv=8, precond="none")
    assert info["status"] == -3, info
    assert bool(torch.isfinite(op.unpack(psi, "f64")).all())
    op.close()


@pytest.fixture(scope="module")
def pair():
    gop, oop, _, _ = make_pair(DIMS, -0.05, 1.7, 0.3, seed=64)
    return gop, oop


def _nan_weights():
    import oracle
    w = oracle.nn_identity_weights()
    w[1][3, 2, 1] = np.nan
    return qdw.nn_weights_tensor(w)


def test_nan_network_hands_the_solve_to_sap(pair):
    """NaN weights: the network's first output is not finite, its GCR column is dropped,
    and with the network-then-SAP preconditioner the solve continues with SAP from the
    same state a SAP-only solve starts from: the same steps and solution."""
    import torch
    gop, oop = pair
    eta_np = syn.gaussian_spinor(DIMS, 65)
    eta = gop.pack(eta_np, "f64")
    kw = dict(res=1e-10, nmx=200, nkv=8, ncy=4, nmr=4, bs=(4, 2, 2, 4), sdtype="f16")
    x_nn = gop.new_field("f64")
    info = qdw.sap_gcr_solve(gop, eta, x_nn, precond="nn_sap", nn_weights=_nan_weights(), **kw)
    x_sap = gop.new_field("f64")
    ref = qdw.sap_gcr_solve(gop, eta, x_sap, precond="sap", **kw)
    assert info["status"] > 0 and info["status"] == ref["status"], (info, ref)
    assert info["nreset"] == ref["nreset"] + 1  # the restart that dropped the column
    x = gop.unpack(x_nn, "f64").cpu().numpy()
    assert np.linalg.norm(x - gop.unpack(x_sap, "f64").cpu().numpy()) <= 1e-12 * np.linalg.norm(x)
    assert np.linalg.norm(eta_np - oop.dw(x)) <= 1.01e-10 * np.linalg.norm(eta_np)


def test_nan_network_alone_ends_with_status_minus_3(pair):
    import torch
    gop, _ = pair
    eta = gop.pack(syn.gaussian_spinor(DIMS, 66), "f64")
    psi = gop.new_field("f64")
    info = qdw.sap_gcr_solve(gop, eta, psi, res=1e-10, nmx=50, nkv=8, precond="nn",
                             nn_weights=_nan_weights())
    assert info["status"] == -3
    assert bool(torch.isfinite(gop.unpack(psi, "f64")).all())


def test_operator_memory_is_a_torch_allocation():
    """The operator's arrays live in one torch tensor of qdw_op_device_bytes bytes: torch's
    allocator accounts for all of them, and they go back to it when the operator closes."""
    import torch
    dims = (16, 8, 8, 8)
    su3, th = syn.gauge_field(dims, 0.3, 0.1, 67)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    op = qdw.Op(dims, su3, th, -0.05, 1.7, -1)
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated() - before
    V = int(np.prod(dims))
    assert op.device_bytes >= V * (4 * 224 + 2 * 1152 + 880)
    assert op.device_bytes <= grown <= op.device_bytes + 4096
    op.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - before <= 4096
