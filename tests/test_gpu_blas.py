"""Fused BLAS-1 through the C ABI against numpy in FP64 (tolerance 1e-14 relative for
FP64 fields; for lower-precision storage the comparison is with the rounded values the
field holds, so the FP64 reduction must agree to 1e-13) and bitwise reproducibility."""
import numpy as np
import pytest

from paper_2202_07388_amd import qdw
from paper_2202_07388_amd import synthetic as syn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[(4, 4, 4, 4), (6, 4, 4, 6), (16, 8, 8, 8)])
def setup(request):
    dims = request.param
    su3, th = syn.unit_gauge_field(dims)
    op = qdw.Op(dims, su3, th, 0.0, 1.0)
    a = syn.gaussian_spinor(dims, 1)
    b = syn.gaussian_spinor(dims, 2)
    return dims, op, a, b


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_norm_dot_axpby(setup, prec):
    dims, op, a, b = setup
    xa, xb = op.pack(a, prec), op.pack(b, prec)
    ra = op.unpack(xa, prec).cpu().numpy()   # what the field holds
    rb = op.unpack(xb, prec).cpu().numpy()
    n = qdw.norm2(op, xa, prec)
    assert abs(n - np.vdot(ra, ra).real) <= 1e-13 * n
    d = qdw.cdot(op, xa, xb, prec)
    want = np.vdot(ra, rb)
    assert abs(d - want) <= 1e-13 * np.sqrt(np.vdot(ra, ra).real * np.vdot(rb, rb).real)
    qdw.axpby(op, 0.5, xa, -2.0, xb, prec)
    got = op.unpack(xb, prec).cpu().numpy()
    ref = 0.5 * ra - 2.0 * rb
    tol = {"f64": 1e-15, "f32": 2e-7, "f16": 2e-3, "bf16": 1.6e-2}[prec]
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


def test_reductions_bitwise_reproducible(setup):
    dims, op, a, b = setup
    xa, xb = op.pack(a), op.pack(b)
    assert len({qdw.norm2(op, xa) for _ in range(5)}) == 1
    assert len({qdw.cdot(op, xa, xb) for _ in range(5)}) == 1
