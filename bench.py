"""Benchmark of the Wilson-clover operator and its solvers on one MI355X.

Timed steps (the `value`): one application of D in FP64 at 32^3 x 64 (V = 2,097,152
sites), near-identity SU(3) x U(1) links (eps = 0.3, U(1) eps = 0.1), m0 = -0.05,
c_sw = 1.7, antiperiodic time, Gaussian source; throughput in GB/s of algorithmic HBM
bytes (1376 B per site: spinor in and out, 4 links of 12 + 1 reals, 72 clover reals,
each read once), inputs resident in HBM.

Also reported, each timed on its own outside the K steps:
  * D in FP32 and FP16 storage, D^+ in FP64, and FP64 D on 4 fields in one launch;
  * the link-storage control: FP64 D and D^+ with full 3x3 links (18 reals) against the
    two-row storage, both in the one-lane-per-site form;
  * the 32^3 x 64 normal-equation solve to FP64 true residual 1e-10: plain FP64 CG
    against FP32, FP16 and BF16 regular steps with FP64 reset steps, and the BF16 -> FP32
    -> FP64 precision cascade; and the even-odd reduced normal equations D^+ D^ psi_e =
    eta_e (FP64, FP32 and FP16 inner, and the cascade), which the solver of the full
    equations is compared with;
  * the 24^3 x 48 solve of D psi = eta to 1e-10 (eps = 0.35, m0 = -0.08): plain FP64 GCR
    against SAP-preconditioned GCR (4^4 blocks, 5 cycles, 4 MR steps, FP16 and FP32), the
    same with even-odd reduced block solves (FP16) and adaptive SAP (at most 20 cycles and
    20 MR steps, alpha 0.9 and 0.7, FP16), and SAP applications alone (plain and with
    even-odd reduced blocks, FP16 and FP32 storage);
  * the learned preconditioner: trained on the GPU on 2000 residual/error pairs from
    plain FP64 GCR solves on four 16^3 x 32 fields (eps = 0.3, m0 = -0.05), then used as
    the flexible-GCR preconditioner on the 32^3 x 64 field against SAP-GCR (plain and with
    even-odd reduced blocks) and plain GCR, all to 1e-10;
  * a batch of 40 right-hand sides over three lattices of different volumes (16^3 x 32
    with 12 point sources, one per spin and colour; 24^3 x 48 with 4 Gaussian sources;
    8^3 x 16 with 24 Gaussian sources; three independent fields, eps = 0.3, m0 = -0.05),
    mixed-precision SAP-GCR to 1e-10 as one captured batch plan (one or two GCR restart
    cycles per graph launch, one host wait per launch) against the same 40 solves one
    after another, with plain and with even-odd reduced SAP blocks, and the D-kernel
    shape the autotuner picked per lattice;
  * the FP64 oracle timed on the host (cpu_baseline): D at 32^3 x 64 on all host cores and
    on one core, and CGNE / GCR / SAP-GCR solves at small lattices beside the GPU's.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-solves]
                       [--legs links,multi,cgne,nn,gcr,sap,batch] [--autotune] [--calibrate]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DIMS = (64, 32, 32, 32)
M0, CSW, EPS, EPS_U1 = -0.05, 1.7, 0.3, 0.1
SEED = 7388 + 10
SAP_DIMS = (48, 24, 24, 24)
SAP_M0, SAP_EPS, SAP_SEED = -0.08, 0.35, 7388 + 20
# D-kernel shapes (ts, nt, pipe, walk, march) at 32^3 x 64, as the autotuner picks them on
# MI355X (profiles/dw_autotune_32c64.md); pinned so that a kernel trace of this script
# holds only the timed shape's launches (--autotune picks them live)
PINNED_SHAPES = {"f64": (64, 32, 0, 0, 1), "f32": (128, 16, 1, 0, 1), "f16": (128, 2, 0, 0, 0)}
# algorithmic bytes per site of one application of D (each datum read once)
BYTES_PER_SITE = {"f64": 1376, "f32": 688, "f16": 344}
# HBM traffic measured with rocprofv3 counters for the FP64 kernel (profiles/); reported
# only while the kernel sources are the ones it was measured on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dw_f64_32c64_traffic.json")
KERNEL_SOURCES = ["paper_2202_07388_amd/csrc/dirac.hip", "paper_2202_07388_amd/csrc/dirac_core.h",
                  "paper_2202_07388_amd/csrc/qdw_internal.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(shape):
    """HBM bytes per launch of the FP64 D kernel from the committed counter runs, while the
    kernel sources and the shape are the ones they were taken with."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or list(t.get("shape", [])) != list(shape):
        return None
    return t.get("bytes_per_launch")


def time_launches(fn, n):
    """Average duration of n launches of fn, bracketed by HIP events recorded on the stream
    the library launches on (torch's current stream)."""
    import torch
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(n):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / n


CPU_CGNE_DIMS, CPU_SAP_DIMS = (16, 8, 8, 8), (8, 8, 8, 8)


def cpu_baseline(su3, th, psi):
    """The FP64 oracle (C site loops with OpenMP, -O3 -march=native, built on this host),
    timed on this host: D at the full 32^3 x 64 on all host cores (median of 5) and on one
    core (one application), clover build excluded; and two solves to rel. residual 1e-10
    at smaller lattices of the same recipes, with the GPU timed on the same solves:
    CGNE on D^+ D at 16 x 8^3 (eps 0.3, m0 -0.05) and flexible GCR at 8^4 (eps 0.35,
    m0 -0.08), plain and with SAP (4^4 blocks, 5 cycles, 4 MR steps)."""
    import oracle
    from paper_2202_07388_amd import qdw
    from paper_2202_07388_amd import synthetic as syn
    oracle.use_native_build()
    nproc = len(os.sched_getaffinity(0))
    oracle.set_threads(nproc)
    cores = oracle.max_threads()
    V = int(np.prod(DIMS))
    op = oracle.Operator(DIMS, su3, th, M0, CSW, -1)
    op.dw(psi)
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        op.dw(psi)
        ts.append(time.perf_counter() - t0)
    d_all = float(np.median(ts))
    oracle.set_threads(1)
    t0 = time.perf_counter()
    op.dw(psi)
    d_one = time.perf_counter() - t0
    oracle.set_threads(cores)
    del op
    solves = {}
    # CGNE, FP64, host and GPU
    su3c, thc = syn.gauge_field(CPU_CGNE_DIMS, EPS, EPS_U1, SEED + 5)
    eta = syn.gaussian_spinor(CPU_CGNE_DIMS, SEED + 5 + 1000)
    oc = oracle.Operator(CPU_CGNE_DIMS, su3c, thc, M0, CSW, -1)
    t0 = time.perf_counter()
    _, st = oracle.cgne(oc, eta, 1e-10, 5000)
    solves["cgne_f64_16x8c3"] = {"host_s": round(time.perf_counter() - t0, 3), "host_steps": st}
    gc = qdw.Op(CPU_CGNE_DIMS, su3c, thc, M0, CSW, -1)
    e = gc.pack(eta)
    for inner in ("f64", "f16"):
        info = qdw.cgne_solve(gc, e, gc.new_field(), res=1e-10, nmx=5000, inner=inner)
        solves["cgne_f64_16x8c3"]["gpu_%s_inner_s" % inner] = round(info["t_sec"], 4)
        solves["cgne_f64_16x8c3"]["gpu_%s_inner_steps" % inner] = info["n_steps"]
    gc.close()
    # flexible GCR, plain and SAP-preconditioned
    su3s, ths = syn.gauge_field(CPU_SAP_DIMS, SAP_EPS, EPS_U1, SEED + 15)
    eta = syn.gaussian_spinor(CPU_SAP_DIMS, SEED + 15 + 1000)
    os_ = oracle.Operator(CPU_SAP_DIMS, su3s, ths, SAP_M0, CSW, -1)
    gs = qdw.Op(CPU_SAP_DIMS, su3s, ths, SAP_M0, CSW, -1)
    e = gs.pack(eta)
    bs = (4, 4, 4, 4)
    for name, M, kw in (("gcr_plain_8c4", None, dict(precond="none")),
                        ("sap_gcr_8c4", lambda v: oracle.sap(os_, v, bs, 5, 4),
                         dict(precond="sap", sdtype="f32", ncy=5, nmr=4, bs=bs))):
        t0 = time.perf_counter()
        _, st = oracle.fgcr(os_, eta, 1e-10, 5000, 16, M)
        rec = {"host_s": round(time.perf_counter() - t0, 3), "host_steps": st}
        info = qdw.sap_gcr_solve(gs, e, gs.new_field(), res=1e-10, nmx=5000, nkv=16, **kw)
        rec.update(gpu_s=round(info["t_sec"], 4), gpu_steps=info["n_steps"])
        solves[name] = rec
    gs.close()
    return {"value": round(BYTES_PER_SITE["f64"] * V / d_all / 1e9, 3), "unit": "GB/s",
            "cores": cores, "kind": "oracle",
            "sample": "oracle D (FP64, C with OpenMP over sites, -O3 -march=native) at the full "
                      "32^3x64 on %d threads, median of 5 applications (%.3f s each), clover "
                      "build excluded; solves at 16x8^3 (CGNE) and 8^4 (GCR) as listed"
                      % (cores, d_all),
            "one_core_GB_s": round(BYTES_PER_SITE["f64"] * V / d_one / 1e9, 3),
            "one_core_s": round(d_one, 3),
            "host_nproc": nproc,
            "solves": solves}


def solve_record(info):
    return {"s": round(info["t_sec"], 4), "steps": info["n_steps"], "status": info["status"],
            "resets_or_restarts": info["nreset"], "rel_res_true": info["rel_res_true"],
            "dw_fp64": info["n_dw_hi"], "dw_low": info["n_dw_lo"]}


def links_control(op, qdw, psi, shape=(128, 4, 0, 0, 0)):
    """The link-storage control at 32^3 x 64: FP64 D and D^+ with the links read as full 3x3
    matrices (18 reals) against the two-row storage (12 reals + det U, third row rebuilt in
    the kernel), both in the one-lane-per-site form with a plain hop loop on the same walk
    (the only form the control exists in). Nominal bytes per site 1536 and 1376. The
    operator's FP64 shape is restored afterwards."""
    keep = qdw.get_dw_shape(op, "f64")
    x, y = op.pack(psi, "f64"), op.new_field("f64")
    qdw.set_full_links(op)
    rec = {"shape": list(shape)}
    try:
        qdw.set_dw_shape(op, "f64", *shape)
        for name, fn, per_site in (
                ("two_row_13", lambda: qdw.dw_apply(op, x, y, "f64"), 1376),
                ("full_18", lambda: qdw.dw_apply_full_links(op, x, y), 1536),
                ("two_row_13_dag", lambda: qdw.dw_dag_apply(op, x, y, "f64"), 1376),
                ("full_18_dag", lambda: qdw.dw_apply_full_links(op, x, y, dagger=True), 1536)):
            for _ in range(5):
                fn()
            d = time_launches(fn, 50)
            rec[name] = {"ms": round(d * 1e3, 4), "GB_s_nominal": round(per_site * op.V / d / 1e9, 1)}
    finally:
        qdw.set_dw_shape(op, "f64", *keep)
        op._full_links = None
    log("  link-storage control: %s" % rec)
    return rec


def multi_rhs(op, qdw, psi, n=4):
    """D on n FP64 fields in one launch (links and clover read once for all of them), in the
    shape the autotuner picks for n fields: per-field time and the rate in algorithmic
    bytes. The operator's FP64 shape is restored afterwards."""
    keep = qdw.get_dw_shape(op, "f64")
    xs = [op.pack(psi * (1.0 + 0.25 * r), "f64") for r in range(n)]
    ys = [op.new_field("f64") for _ in range(n)]
    try:
        shape = qdw.autotune(op, "f64", n).split(";")[0]
        f = lambda: qdw.dw_apply_multi(op, xs, ys, "f64")
        for _ in range(3):
            f()
        d = time_launches(f, 20)
    finally:
        qdw.set_dw_shape(op, "f64", *keep)
    per_site = n * 2 * 192 + 4 * 104 + 576
    rec = {"rhs": n, "ms": round(d * 1e3, 4), "ms_per_field": round(d * 1e3 / n, 4),
           "bytes_per_site": per_site, "GB_s": round(per_site * op.V / d / 1e9, 1),
           "shape": shape}
    log("  multi-RHS D: %s" % rec)
    del xs, ys
    return rec


def cgne_solves(op, qdw, psi):
    """Plain FP64 CG against mixed precision, D^+ D psi = eta to 1e-10 (32^3 x 64). The
    mixed legs keep the search direction across resets (reliable updates after a drop of
    10); the *_paper_reset legs restart CG at every reset, triggered after a drop of
    10 eps of the working type (Sec. 2, Fig. 1)."""
    eta = op.pack(psi, "f64")
    out = {}
    for name, kw in (("f64", dict(inner="f64")), ("f32", dict(inner="f32")),
                     ("f16", dict(inner="f16")), ("bf16", dict(inner="bf16")),
                     ("f32_paper_reset", dict(inner="f32", keep_p=False)),
                     ("f16_paper_reset", dict(inner="f16", keep_p=False)),
                     ("bf16_paper_reset", dict(inner="bf16", keep_p=False)),
                     ("cascade_bf16_f32_f64", dict(cascade=True)),
                     ("schur_f64", dict(inner="f64", schur=True)),
                     ("schur_f32", dict(inner="f32", schur=True)),
                     ("schur_f16", dict(inner="f16", schur=True)),
                     ("schur_cascade_bf16_f32_f64", dict(cascade=True, schur=True))):
        x = op.new_field("f64")
        info = qdw.cgne_solve(op, eta, x, res=1e-10, nmx=20000, **kw)
        out[name] = solve_record(info)
        log("  cgne %s: %s" % (name, out[name]))
    return out


def gcr_solves(qdw, syn):
    """Plain FP64 GCR against SAP-GCR, D psi = eta to 1e-10 (24^3 x 48)."""
    su3, th = syn.gauge_field(SAP_DIMS, SAP_EPS, EPS_U1, SAP_SEED)
    op = qdw.Op(SAP_DIMS, su3, th, SAP_M0, CSW, -1)
    del su3, th
    eta = op.pack(syn.gaussian_spinor(SAP_DIMS, SAP_SEED + 1000), "f64")
    out = {"dw_shape": qdw.autotune(op, "f64", 1).split(";")[0]}  # the outer FP64 D
    base = dict(ncy=5, nmr=4)
    adaptive = dict(precond="sap_adaptive", sdtype="f16", ncy=20, nmr=20)
    for name, kw in (("plain_fp64", dict(base, precond="none")),
                     ("sap_fp16", dict(base, precond="sap", sdtype="f16")),
                     ("sap_fp32", dict(base, precond="sap", sdtype="f32")),
                     ("sap_eo_fp16", dict(base, precond="sap_eo", sdtype="f16")),
                     ("sap_adaptive_fp16_alpha0.9", dict(adaptive, alpha=0.9)),
                     ("sap_adaptive_fp16_alpha0.7", dict(adaptive, alpha=0.7))):
        x = op.new_field("f64")
        info = qdw.sap_gcr_solve(op, eta, x, res=1e-10, nmx=5000, nkv=16, bs=(4, 4, 4, 4), **kw)
        out[name] = solve_record(info)
        log("  gcr %s: %s" % (name, out[name]))
    op.close()
    return out


def sap_sweeps(qdw, syn):
    """SAP applications at 24^3 x 48 (eps 0.35, m0 -0.08; 4^4 blocks, 5 cycles, 4 MR steps):
    plain and even-odd reduced block solves, FP16 and FP32 storage, each timed over 10
    applications after 3 warm-up ones (a kernel trace of this leg holds only these)."""
    import torch
    su3, th = syn.gauge_field(SAP_DIMS, SAP_EPS, EPS_U1, SAP_SEED)
    op = qdw.Op(SAP_DIMS, su3, th, SAP_M0, CSW, -1)
    del su3, th
    rho = op.pack(syn.gaussian_spinor(SAP_DIMS, SAP_SEED + 1000), "f64")
    phi = op.new_field("f64")
    out = {}
    for eo in (False, True):
        for prec in ("f16", "f32"):
            f = lambda: qdw.sap_apply(op, rho, phi, 5, 4, (4, 4, 4, 4), prec, eo=eo)
            for _ in range(3):
                f()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(10):
                f()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / 10 * 1e3
            out["%s_%s" % ("eo" if eo else "plain", prec)] = {"ms_per_application": round(ms, 4)}
            log("  sap %s %s: %.3f ms per application" % ("eo" if eo else "plain", prec, ms))
    op.close()
    return out


NN_DIMS = (32, 16, 16, 16)
NN_FIELDS, NN_SOURCES, NN_STEPS, NN_PAIRS = 4, 6, 100, 2000


def learned_preconditioner(qdw, syn, op, psi):
    """Train the network on solver pairs at 16^3x32; evaluate it as the FGCR
    preconditioner on the 32^3x64 operator against SAP-GCR and plain GCR."""
    import torch
    from paper_2202_07388_amd import nn_train
    t0 = time.perf_counter()
    groups = []
    for f in range(NN_FIELDS):
        seed = 7388 + 40 + f
        su3, th = syn.gauge_field(NN_DIMS, EPS, EPS_U1, seed)
        top = qdw.Op(NN_DIMS, su3, th, M0, CSW, -1)
        del su3, th
        etas = [top.pack(syn.gaussian_spinor(NN_DIMS, seed + 1000 + k)) for k in range(NN_SOURCES)]
        r, e = nn_train.solver_pairs(top, etas, NN_STEPS, store="bf16")
        groups.append((top, r, e))
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    # keep NN_PAIRS pairs, drawn evenly from the fields
    rng = np.random.Generator(np.random.PCG64(7388))
    per = NN_PAIRS // NN_FIELDS
    for f, (top, r, e) in enumerate(groups):
        keep = sorted(rng.permutation(len(r))[:per])
        groups[f] = (top, [r[i] for i in keep], [e[i] for i in keep])
    npairs = sum(len(g[1]) for g in groups)
    log("  nn: %d pairs in %.1f s" % (npairs, t_pairs))
    t0 = time.perf_counter()
    w, losses = nn_train.train(None, None, None, "bf16", epochs=3, batch=16, lr=5e-3, m0=M0,
                               groups=groups)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    for g in groups:
        g[0].close()
    del groups
    log("  nn: trained %d steps in %.1f s, loss %.4f -> %.4f" % (
        len(losses), t_train, float(np.mean(losses[:10])), float(np.mean(losses[-10:]))))
    eta = op.pack(psi, "f64")
    out = {"pairs": npairs, "train_steps": len(losses),
           "s_pairs": round(t_pairs, 2), "s_train": round(t_train, 2),
           "loss_first10": round(float(np.mean(losses[:10])), 5),
           "loss_last10": round(float(np.mean(losses[-10:])), 5)}
    for name, kw in (("plain_fp64", dict(precond="none")),
                     ("nn", dict(precond="nn", nn_weights=w)),
                     ("nn_then_sap_fp16", dict(precond="nn_sap", nn_weights=w, sdtype="f16")),
                     ("sap_fp16", dict(precond="sap", sdtype="f16")),
                     ("sap_eo_fp16", dict(precond="sap_eo", sdtype="f16"))):
        x = op.new_field("f64")
        info = qdw.sap_gcr_solve(op, eta, x, res=1e-10, nmx=5000, nkv=16, ncy=5, nmr=4,
                                 bs=(4, 4, 4, 4), **kw)
        out[name] = solve_record(info)
        log("  gcr 32c64 %s: %s" % (name, out[name]))
        del x
    return out


BATCH = (((32, 16, 16, 16), "point", 12, 7388 + 31), ((48, 24, 24, 24), "gauss", 4, 7388 + 32),
         ((16, 8, 8, 8), "gauss", 24, 7388 + 33))


def batched_solves(qdw, syn):
    """40 right-hand sides over three lattices: one batched SAP-GCR against 40 single solves,
    with plain SAP and with even-odd reduced SAP blocks."""
    ops, etas, shapes = [], [], {}
    for dims, kind, n, seed in BATCH:
        su3, th = syn.gauge_field(dims, EPS, EPS_U1, seed)
        op = qdw.Op(dims, su3, th, M0, CSW, -1)
        del su3, th
        name = "%dc%d" % (dims[1], dims[0])
        shapes[name] = qdw.autotune(op, "f64", n).split(";")[0]
        for r in range(n):
            src = (syn.point_spinor(dims, r // 3, r % 3, 0) if kind == "point"
                   else syn.gaussian_spinor(dims, seed + 1000 + r))
            ops.append(op)
            etas.append(op.pack(src, "f64"))
    out = {}
    for precond in ("sap", "sap_eo"):
        out[precond] = batched_run(qdw, ops, etas, shapes, precond)
    for o in set(ops):
        o.close()
    return out


def batched_run(qdw, ops, etas, shapes, precond):
    """The batch as captured plans (qdw.Batch) of 1 and 2 restart cycles per graph launch:
    capture time, a warm-up solve, then one timed solve each; against the same solves one
    after another."""
    import torch
    kw = dict(res=1e-10, nmx=2000, nkv=16, ncy=5, nmr=4, bs=(4, 4, 4, 4), sdtype="f16",
              precond=precond)
    plans = {}
    for cycles in (1, 2):
        plan = qdw.Batch(ops, cycles=cycles, **kw)
        psis = [o.new_field("f64") for o in ops]
        plan.solve(etas, psis)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos, launches = plan.solve(etas, psis)
        torch.cuda.synchronize()
        plans[cycles] = (time.perf_counter() - t0, launches, plan.capture_ms, infos)
        plan.close()
        del psis
    t0 = time.perf_counter()
    single = []
    for o, e in zip(ops, etas):
        x = o.new_field("f64")
        single.append(qdw.sap_gcr_solve(o, e, x, **kw))
        del x
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    best = min(plans, key=lambda c: plans[c][0])
    t_batch, _, _, infos = plans[best]
    per = {}
    i = 0
    for dims, kind, n, seed in BATCH:
        name = "%dc%d" % (dims[1], dims[0])
        inf = infos[i:i + n]
        per[name] = {"rhs": n, "source": kind,
                     "steps": [x["n_steps"] for x in inf],
                     "max_rel_res_true": max(x["rel_res_true"] for x in inf),
                     "all_converged": all(x["status"] > 0 for x in inf),
                     "same_steps_as_single": all(a["status"] == b["status"]
                                                 for a, b in zip(inf, single[i:i + n])),
                     "dw_shape": shapes[name]}
        i += n
    site_rhs = sum(int(np.prod(d)) * n for d, _, n, _ in BATCH)
    rec = {"rhs": len(ops), "site_rhs": site_rhs, "s_batched": round(t_batch, 4),
           "cycles_per_launch": best,
           "plans": {str(c): {"s": round(v[0], 4), "graph_launches": v[1],
                              "capture_ms": round(v[2], 2)} for c, v in plans.items()},
           "s_sequential_single": round(t_seq, 4),
           "speedup": round(t_seq / t_batch, 3), "lattices": per,
           "settings": "SAP-GCR nkv 16, 4^4 blocks, ncy 5, nmr 4, FP16 SAP storage, res 1e-10, "
                       "precond %s; one host wait per graph launch" % precond}
    log("  batched %s: %s" % (precond, json.dumps(rec)))
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solves", action="store_true")
    ap.add_argument("--no-nn", action="store_true", help="skip training the learned preconditioner")
    ap.add_argument("--legs", default="links,multi,cgne,nn,gcr,sap,batch",
                    help="comma-separated legs to run after the D timing (links: the "
                         "full-matrix link control; multi: D on 4 fields in one launch; "
                         "cgne, nn, gcr, batch: solves; sap: SAP applications); kernel "
                         "traces of one leg use this")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the 32^3x64 D-kernel shapes with the autotuner instead of the "
                         "pinned ones (its own launches then join any kernel trace)")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a plain elementwise kernel that reads and writes 1 GiB "
                         "(3 launches), to scale hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2202_07388_amd import qdw
    from paper_2202_07388_amd import synthetic as syn

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    qdw.load()
    log("generating the 32^3x64 gauge field ...")
    t0 = time.time()
    su3, th = syn.gauge_field(DIMS, EPS, EPS_U1, SEED)
    psi = syn.gaussian_spinor(DIMS, SEED + 1000)
    log("  %.1f s; creating the operator" % (time.time() - t0))
    op = qdw.Op(DIMS, su3, th, M0, CSW, -1)
    if args.no_cpu_baseline:
        del su3, th
    V = op.V
    if args.autotune:
        log("autotuning the D kernel ...")
        tuned = {}
        for p in ("f64", "f32", "f16"):
            rep = qdw.autotune(op, p, 1)
            log("  autotune %s: %s" % (p, rep))
            tuned[p] = rep.split(";")[0]
    else:
        for p, shape in PINNED_SHAPES.items():
            qdw.set_dw_shape(op, p, *shape)
        tuned = {p: "pinned ts,nt,pipe,walk,march = %s" % (shape,) for p, shape in PINNED_SHAPES.items()}
    log("  D-kernel shapes: %s" % tuned)
    fields = {}
    for prec in ("f64", "f32", "f16"):
        fields[prec] = (op.pack(psi, prec), op.new_field(prec))
    torch.cuda.synchronize()

    x64, y64 = fields["f64"]
    # the other precisions and D^+ first: the timed FP64 launches then run on a GPU in its
    # steady state (the first launches after the operator's set-up run up to 7 % slower)
    other = {}
    for prec in ("f32", "f16"):
        x, y = fields[prec]
        f = lambda: qdw.dw_apply(op, x, y, prec)
        for _ in range(10):
            f()
        d = time_launches(f, 100)
        other[prec] = {"ms": round(d * 1e3, 4),
                       "GB_s": round(BYTES_PER_SITE[prec] * V / d / 1e9, 1),
                       "frac_hbm_peak": round(BYTES_PER_SITE[prec] * V / d / 1e9 / HBM_PEAK_GBS, 4)}
    d_dag = time_launches(lambda: qdw.dw_dag_apply(op, x64, y64, "f64"), 50)
    other["f64_dag"] = {"ms": round(d_dag * 1e3, 4),
                        "GB_s": round(BYTES_PER_SITE["f64"] * V / d_dag / 1e9, 1)}

    step = lambda: qdw.dw_apply(op, x64, y64, "f64")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("timing %d FP64 applications" % args.steps)
    # timed region: exactly K steps, bracketed by synchronisation
    torch.cuda.synchronize()
    t_wall0 = time.perf_counter()
    dt = time_launches(step, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall0
    gbs = BYTES_PER_SITE["f64"] * V / dt / 1e9
    del fields

    if args.calibrate:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b

    traffic = measured_traffic(qdw.get_dw_shape(op, "f64"))
    out = {
        "metric": "Dw GB/s (% HBM peak) at 32^3x64; solve s to rel res 1e-10, plain vs chosen",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Wilson-clover D, 32^3x64, FP64, two-row compressed links",
                   "lattice": "32^3x64", "m0": M0, "c_sw": CSW, "eps": EPS,
                   "eps_u1": EPS_U1, "bc_t": "antiperiodic"},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "dw_other_precisions": other,
        "dw_shapes": {p: list(qdw.get_dw_shape(op, p)) for p in ("f64", "f32", "f16")},
        "autotune": tuned,
        "wall_s_timed_region": round(wall, 4),
    }
    legs = set() if args.no_solves else set(args.legs.split(","))
    if args.no_nn:
        legs.discard("nn")
    if legs:
        log("solves: %s ..." % sorted(legs))
    if "links" in legs:
        out["dw_links_control_f64"] = links_control(op, qdw, psi)
    if "multi" in legs:
        out["dw_multi_rhs_f64"] = multi_rhs(op, qdw, psi)
    if "cgne" in legs:
        out["cgne_32c64"] = cgne_solves(op, qdw, psi)
    if "nn" in legs:
        out["learned_precond_32c64"] = learned_preconditioner(qdw, syn, op, psi)
    op.close()
    if "gcr" in legs:
        out["sap_gcr_24c48"] = gcr_solves(qdw, syn)
    if "sap" in legs:
        out["sap_apply_24c48"] = sap_sweeps(qdw, syn)
    if "batch" in legs:
        out["batched_40rhs"] = batched_solves(qdw, syn)
    if not args.no_cpu_baseline:
        log("timing the oracle on the host (bounded sample) ...")
        out["cpu_baseline"] = cpu_baseline(su3, th, psi)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
