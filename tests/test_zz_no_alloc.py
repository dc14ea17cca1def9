"""The allocation-free SAP entry point (static device scratch) against sap_apply.

Both run the same kernels on the same inputs; sap_apply's workspace and the static array
differ only in where the SAP fields live, and every value the application reads is
written first, so the results are bit-identical. Two calls in a row, the second on a
smaller lattice, show that what the first call leaves in the shared array does not leak
into the second.
"""
import ctypes

import numpy as np
import pytest

from paper_2202_07388_amd import qdw
from paper_2202_07388_amd import synthetic as syn

pytestmark = pytest.mark.gpu


def _op(dims, seed):
    su3, th = syn.gauge_field(dims, 0.35, 0.1, seed)
    return qdw.Op(dims, su3, th, -0.08, 1.7, -1)


@pytest.mark.parametrize("sdtype", ["f16", "f32", "bf16"])
def test_noalloc_equals_sap_apply_twice(sdtype):
    import torch
    cases = [((16, 8, 8, 8), (4, 4, 4, 4), 71), ((8, 4, 4, 8), (4, 2, 2, 4), 72)]
    for dims, bs, seed in cases:  # the second call: a smaller lattice
        op = _op(dims, seed)
        rho = op.pack(syn.gaussian_spinor(dims, seed + 1000))
        want = op.new_field()
        qdw.sap_apply(op, rho, want, 3, 4, bs, sdtype)
        got = op.new_field()
        qdw.sap_apply_noalloc(op, rho, got, 3, 4, bs, sdtype)
        assert torch.equal(got, want), (dims, sdtype)
        assert float(torch.abs(op.unpack(got)).max()) > 0
        op.close()


def test_noalloc_rejects_lattices_above_the_maximum():
    """32 x 16^3: the FP16 fields fit the 24 MiB array, the FP32 ones (38 MB) do not."""
    dims = (32, 16, 16, 16)
    op = _op(dims, 73)
    lib = qdw.load()
    cap = lib.qdw_sap_noalloc_max_bytes()
    assert cap == 24 << 20
    assert lib.qdw_sap_workspace_bytes(op.handle, qdw.PREC["f32"]) > cap
    assert lib.qdw_sap_workspace_bytes(op.handle, qdw.PREC["f16"]) <= cap
    rho = op.pack(syn.gaussian_spinor(dims, 74))
    phi = op.new_field()
    with pytest.raises(qdw.QdwError, match="static maximum"):
        qdw.sap_apply_noalloc(op, rho, phi, 1, 2, (4, 4, 4, 4), "f32")
    qdw.sap_apply_noalloc(op, rho, phi, 1, 2, (4, 4, 4, 4), "f16")
    want = op.new_field()
    qdw.sap_apply(op, rho, want, 1, 2, (4, 4, 4, 4), "f16")
    import torch
    assert torch.equal(phi, want)
    op.close()
