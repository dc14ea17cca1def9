"""Several right-hand sides and lattices at once: the multi-right-hand-side D, the D-kernel
shapes and their autotuner, and the batched flexible GCR replayed as a HIP graph.

Bars: D on several fields in one launch equals D on each field bit for bit (every site's
arithmetic is the same, only the workgroup schedule changes), and so does D under every
kernel shape; against the FP64 oracle D stays within 1e-13 (FP64) and 2e-6 (FP32). A
batched solve takes the same steps as the single solve of the same system: same status,
restart count and (within the rounding of the device-side triangular solve) the same
solution, so solutions agree to 1e-9 relative while both reach the FP64 true residual
1e-10, which is checked here with the oracle's D.
"""
import numpy as np
import pytest

import oracle
from paper_2202_07388_amd import qdw
from paper_2202_07388_amd import synthetic as syn
from gpu_util import make_pair, maxrel, rel

pytestmark = pytest.mark.gpu

DIMS_RAGGED = (6, 4, 6, 10)  # T not a power of two, S = 120: tiles of 64 / 128 sites are ragged


@pytest.fixture(scope="module")
def ragged():
    gop, oop, _, _ = make_pair(DIMS_RAGGED, -0.05, 1.7, 0.3, seed=91)
    srcs = [syn.gaussian_spinor(DIMS_RAGGED, 300 + r) for r in range(5)]
    return gop, oop, srcs


@pytest.mark.parametrize("dims", [(6, 4, 6, 10), (4, 4, 4, 4)])
def test_default_shapes(dims):
    """Shapes at creation: FP64 and FP32 march on 64-site tiles (nt = 1 here, where no walk
    chunk gives 512 workgroups), the half-precision storage forms take the plain form on
    128-site tiles in chunks of two slices."""
    su3, th = syn.gauge_field(dims, 0.3, 0.1, 5)
    op = qdw.Op(dims, su3, th, -0.05, 1.7, -1)
    try:
        assert qdw.get_dw_shape(op, "f64") == (64, 1, 0, 0, 1)
        assert qdw.get_dw_shape(op, "f32") == (64, 1, 1, 0, 1)
        for prec in ("f16", "bf16"):
            assert qdw.get_dw_shape(op, prec) == (128, 2, 0, 0, 0)
    finally:
        op.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_multi_rhs_equals_single(ragged, prec):
    import torch
    gop, oop, srcs = ragged
    xs = [gop.pack(s, prec) for s in srcs]
    outs = [gop.new_field(prec) for _ in srcs]
    qdw.dw_apply_multi(gop, xs, outs, prec)
    for x, o in zip(xs, outs):
        one = gop.new_field(prec)
        qdw.dw_apply(gop, x, one, prec)
        assert torch.equal(one, o)


def test_multi_rhs_matches_oracle(ragged):
    gop, oop, srcs = ragged
    xs = [gop.pack(s, "f64") for s in srcs]
    outs = [gop.new_field("f64") for _ in srcs]
    qdw.dw_apply_multi(gop, xs, outs, "f64")
    for s, o in zip(srcs, outs):
        assert maxrel(gop.unpack(o, "f64").cpu().numpy(), oop.dw(s)) <= 1e-13


def test_multi_rhs_rejects_aliasing(ragged):
    gop, oop, srcs = ragged
    xs = [gop.pack(s, "f64") for s in srcs[:2]]
    with pytest.raises(qdw.QdwError, match="alias"):
        qdw.dw_apply_multi(gop, xs, [xs[1], gop.new_field("f64")], "f64")


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 2e-6), ("f16", 2e-2)])
@pytest.mark.parametrize("ts", [64, 128])
@pytest.mark.parametrize("nt", [1, 2, 3, 6])
@pytest.mark.parametrize("pipe,march", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("walk", [0, 1])
def test_every_shape_gives_the_same_d(ragged, prec, tol, ts, nt, pipe, march, walk):
    """Workgroup size, walk chunk and tile order change only the schedule: bit-identical
    results within one kernel form. The forms (plain, pipelined, marching) are separately
    compiled code (the compiler may fuse multiply-adds differently), so across forms the
    bar is the oracle's. The marching form hands the time hops over through LDS; nt = 1
    and 6 (= T) are its edge cases (no hand-over; the whole time extent, wrapping)."""
    import torch
    gop, oop, srcs = ragged
    if march and prec == "f64" and ts == 128:
        with pytest.raises(qdw.QdwError, match="LDS"):
            qdw.set_dw_shape(gop, prec, ts, nt, pipe, walk, march)
        return
    keep = qdw.get_dw_shape(gop, prec)
    x = gop.pack(srcs[0], prec)
    try:
        qdw.set_dw_shape(gop, prec, 64, 1, pipe, 0, march)
        ref = gop.new_field(prec)
        qdw.dw_apply(gop, x, ref, prec)
        qdw.set_dw_shape(gop, prec, ts, nt, pipe, walk, march)
        assert qdw.get_dw_shape(gop, prec) == (ts, nt, pipe, walk, march)
        out = gop.new_field(prec)
        qdw.dw_apply(gop, x, out, prec)
        dag = gop.new_field(prec)
        qdw.dw_dag_apply(gop, x, dag, prec)
    finally:
        qdw.set_dw_shape(gop, prec, *keep)
    assert torch.equal(out, ref)
    assert maxrel(gop.unpack(out, prec).cpu().numpy(), oop.dw(srcs[0])) <= tol
    assert maxrel(gop.unpack(dag, prec).cpu().numpy(), oop.dw_dag(srcs[0])) <= tol


@pytest.mark.parametrize("march", [0, 1])
def test_multi_rhs_in_every_form(ragged, march):
    """Several right-hand sides in one launch of either form equal the single launches."""
    import torch
    gop, oop, srcs = ragged
    keep = qdw.get_dw_shape(gop, "f64")
    try:
        qdw.set_dw_shape(gop, "f64", 64, 2, 1, 1, march)
        xs = [gop.pack(s, "f64") for s in srcs]
        outs = [gop.new_field("f64") for _ in srcs]
        qdw.dw_apply_multi(gop, xs, outs, "f64")
        for s_, x, o in zip(srcs, xs, outs):
            one = gop.new_field("f64")
            qdw.dw_apply(gop, x, one, "f64")
            assert torch.equal(one, o)
            assert maxrel(gop.unpack(o, "f64").cpu().numpy(), oop.dw(s_)) <= 1e-13
    finally:
        qdw.set_dw_shape(gop, "f64", *keep)


def test_bad_shapes_rejected(ragged):
    gop, _, _ = ragged
    for ts, nt, pipe, walk, march in [(96, 1, 0, 0, 0), (128, 4, 0, 0, 0), (64, 1, 2, 0, 0),
                                      (64, 0, 1, 0, 0), (64, 1, 1, 2, 0), (64, 12, 1, 0, 0),
                                      (64, 1, 1, 0, 2)]:
        with pytest.raises(qdw.QdwError, match="shape"):
            qdw.set_dw_shape(gop, "f64", ts, nt, pipe, walk, march)


def test_autotune_picks_a_valid_shape_and_keeps_results(ragged):
    import torch
    gop, oop, srcs = ragged
    x = gop.pack(srcs[1], "f64")
    before = gop.new_field("f64")
    qdw.dw_apply(gop, x, before, "f64")
    rep = qdw.autotune(gop, "f64", nrhs=3)
    # one workgroup per slice: ts {64,128} x nt {1,2} (the powers of two dividing T = 6) x
    # pipe {0,1} x walk {0,1}; marching (FP64 at ts 64 only): nt {1,2} x pipe x walk
    assert "best" in rep and rep.count("[") == 2 * 2 * 2 * 2 + 2 * 2 * 2
    ts, nt, pipe, walk, march = qdw.get_dw_shape(gop, "f64")
    assert ts in (64, 128) and nt in (1, 2) and pipe in (0, 1) and walk in (0, 1)
    assert "ts=%d nt=%d pipe=%d walk=%d march=%d" % (ts, nt, pipe, walk, march) in rep
    after = gop.new_field("f64")
    qdw.dw_apply(gop, x, after, "f64")
    assert maxrel(gop.unpack(after, "f64").cpu().numpy(), oop.dw(srcs[1])) <= 1e-13
    assert maxrel(gop.unpack(after, "f64").cpu().numpy(),
                  gop.unpack(before, "f64").cpu().numpy()) <= 1e-14


# ---------------------------------------------------------------- batched flexible GCR

@pytest.fixture(scope="module")
def batch():
    """Three lattices of different volumes; 3 + 2 + 1 right-hand sides, one a point source."""
    specs = [((8, 8, 8, 8), 101), ((16, 8, 8, 8), 102), ((8, 8, 8, 16), 103)]
    ops = {}
    for dims, seed in specs:
        gop, oop, _, _ = make_pair(dims, -0.05, 1.7, 0.3, seed=seed)
        ops[dims] = (gop, oop)
    probs = []
    d0, d1, d2 = (s[0] for s in specs)
    probs.append((d0, syn.point_spinor(d0, 0, 0, 0)))
    probs.append((d0, syn.gaussian_spinor(d0, 11)))
    probs.append((d1, syn.gaussian_spinor(d1, 12)))
    probs.append((d0, syn.gaussian_spinor(d0, 13)))
    probs.append((d2, syn.gaussian_spinor(d2, 14)))
    probs.append((d1, syn.gaussian_spinor(d1, 15)))
    return ops, probs


def _solve_batched(ops, probs, **kw):
    gops = [ops[d][0] for d, _ in probs]
    etas = [ops[d][0].pack(e, "f64") for d, e in probs]
    psis = [ops[d][0].new_field("f64") for d, _ in probs]
    infos, gms = qdw.sap_gcr_solve_batched(gops, etas, psis, **kw)
    return infos, psis, gms


KW = dict(res=1e-10, nmx=400, nkv=8, ncy=4, nmr=4, bs=(4, 4, 4, 4))


@pytest.mark.parametrize("precond,sdtype", [("sap", "f16"), ("sap", "f32"), ("none", "f32"),
                                            ("sap_eo", "f16")])
def test_batched_equals_single_solves(batch, precond, sdtype):
    ops, probs = batch
    infos, psis, gms = _solve_batched(ops, probs, precond=precond, sdtype=sdtype, **KW)
    assert gms > 0
    for (d, eta), info, psi in zip(probs, infos, psis):
        gop, oop = ops[d]
        e = gop.pack(eta, "f64")
        one = gop.new_field("f64")
        ref = qdw.sap_gcr_solve(gop, e, one, precond=precond, sdtype=sdtype, **KW)
        assert ref["status"] > 0, ref
        assert info["status"] == ref["status"], (d, info, ref)
        assert info["nreset"] == ref["nreset"]
        assert info["rel_res_true"] <= 1e-10
        x = gop.unpack(psi, "f64").cpu().numpy()
        assert rel(x, gop.unpack(one, "f64").cpu().numpy()) <= 1e-9
        r = eta - oop.dw(x)
        assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(eta)


def test_batched_graph_replays_are_deterministic(batch):
    import torch
    ops, probs = batch
    a, pa, _ = _solve_batched(ops, probs, precond="sap", sdtype="f16", **KW)
    b, pb, _ = _solve_batched(ops, probs, precond="sap", sdtype="f16", **KW)
    for ia, ib, xa, xb in zip(a, b, pa, pb):
        assert ia["status"] == ib["status"] and ia["nreset"] == ib["nreset"]
        assert torch.equal(xa, xb)


def test_batched_zero_source_and_nmx(batch):
    """A zero source finishes at once with psi = 0 and leaves the others untouched; nmx
    ends every solve with status -1 after exactly nmx steps, as the single solve does."""
    import torch
    ops, probs = batch
    d0 = probs[0][0]
    mixed = [(d0, np.zeros_like(probs[1][1]))] + probs[1:3]
    infos, psis, _ = _solve_batched(ops, mixed, precond="sap", sdtype="f16", **KW)
    assert infos[0]["status"] == 0 and infos[0]["n_steps"] == 0
    assert float(torch.abs(psis[0]).max()) == 0.0
    assert infos[1]["status"] > 0 and infos[2]["status"] > 0
    kw = dict(KW, nmx=5, nkv=2)
    infos, psis, _ = _solve_batched(ops, probs[:3], precond="sap", sdtype="f16", **kw)
    for (d, eta), info, psi in zip(probs[:3], infos, psis):
        gop, _ = ops[d]
        one = gop.new_field("f64")
        ref = qdw.sap_gcr_solve(gop, gop.pack(eta, "f64"), one, precond="sap", sdtype="f16", **kw)
        assert info["status"] == ref["status"] == -1
        assert info["n_steps"] == 5 and info["nreset"] == ref["nreset"] == 3
        assert rel(gop.unpack(psi, "f64").cpu().numpy(), gop.unpack(one, "f64").cpu().numpy()) <= 1e-9


def test_batched_matches_oracle_fgcr(batch):
    ops, probs = batch
    infos, psis, _ = _solve_batched(ops, probs[:2], precond="sap", sdtype="f16", **KW)
    d, eta = probs[1]
    gop, oop = ops[d]
    xo, st = oracle.fgcr(oop, eta, 1e-11, 3000, 16)
    assert st > 0
    assert rel(gop.unpack(psis[1], "f64").cpu().numpy(), xo) <= 1e-7


def test_batch_plan_reused_across_solves(batch):
    """A captured plan serves several solves: each equals the single solves of its systems
    (same status and restarts, solutions to 1e-9); a plan of several cycles per launch
    gives bit-identical solutions to a plan of one cycle, and finishes in
    ceil(cycles needed / cycles per launch) launches -- one when they suffice."""
    import torch
    ops, probs = batch
    gops = [ops[d][0] for d, _ in probs]
    kw = dict(KW, precond="sap", sdtype="f16")
    one_cycle = qdw.Batch(gops, cycles=1, **kw)
    four = qdw.Batch(gops, cycles=4, **kw)
    assert one_cycle.capture_ms > 0 and four.capture_ms > 0
    try:
        for shift in (0, 1):
            srcs = [(d, e if shift == 0 else np.roll(e, 3, axis=0)) for d, e in probs]
            etas = [ops[d][0].pack(e, "f64") for d, e in srcs]
            pa = [ops[d][0].new_field("f64") for d, _ in srcs]
            pb = [ops[d][0].new_field("f64") for d, _ in srcs]
            ia, na = one_cycle.solve(etas, pa)
            ib, nb = four.solve(etas, pb)
            need = max(i["nreset"] for i in ia)
            assert na == need and nb == -(-need // 4)
            for (d, eta), x, y, i, j, e in zip(srcs, pa, pb, ia, ib, etas):
                gop, oop = ops[d]
                assert torch.equal(x, y) and i["status"] == j["status"] > 0
                ref_psi = gop.new_field("f64")
                ref = qdw.sap_gcr_solve(gop, e, ref_psi, **kw)
                assert i["status"] == ref["status"] and i["nreset"] == ref["nreset"]
                xs = gop.unpack(x, "f64").cpu().numpy()
                assert rel(xs, gop.unpack(ref_psi, "f64").cpu().numpy()) <= 1e-9
                assert np.linalg.norm(eta - oop.dw(xs)) <= 1.01e-10 * np.linalg.norm(eta)
    finally:
        one_cycle.close()
        four.close()
