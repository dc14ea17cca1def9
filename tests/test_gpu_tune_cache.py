"""The D-kernel autotune cache on the GPU: the first call tunes and stores the shape, the
second sets the stored shape without tuning, and D in that shape matches the oracle."""
import pytest

from paper_2202_07388_amd import qdw
from paper_2202_07388_amd import synthetic as syn
from gpu_util import make_pair, maxrel

pytestmark = pytest.mark.gpu


def test_autotune_cache_round_trip(tmp_path):
    dims = (8, 8, 8, 8)
    gop, oop, _, _ = make_pair(dims, 0.1, 1.5, 0.3, seed=91)
    path = str(tmp_path / "shapes.json")
    how, shape = qdw.autotune_cached(gop, "f64", 1, path)
    assert how == "tuned" and shape == qdw.get_dw_shape(gop, "f64")
    qdw.set_dw_shape(gop, "f64", 64, 1, 0, 0, 0)
    how2, shape2 = qdw.autotune_cached(gop, "f64", 1, path)
    assert how2 == "cached" and shape2 == shape and qdw.get_dw_shape(gop, "f64") == shape
    psi = syn.gaussian_spinor(dims, 92)
    y = gop.new_field("f64")
    qdw.dw_apply(gop, gop.pack(psi, "f64"), y, "f64")
    assert maxrel(gop.unpack(y).cpu().numpy(), oop.dw(psi)) < 1e-13
