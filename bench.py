"""Benchmark of the Wilson-clover operator on one MI355X.

Workload: 32^3 x 64 lattice (V = 2,097,152 sites), near-identity SU(3) x U(1) links
(eps = 0.3, U(1) eps = 0.1), m0 = -0.05, c_sw = 1.7, antiperiodic time, Gaussian source.
A timed step is one application of D in FP64 with 12-real compressed links (+ U(1)
angle); ``value`` is its throughput in GB/s of algorithmic HBM bytes (1376 B per site:
spinor in and out, 4 links of 13 reals, 72 clover reals, each read once).

Also reported (timed separately, outside the K steps): D in FP32 and FP16 storage, the
solves to FP64 true residual 1e-10 (plain FP64 against the mixed-precision / SAP
forms), and the FP64 oracle timed on the host's cores on a bounded sample.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
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
# algorithmic bytes per site of one application of D (each datum read once)
BYTES_PER_SITE = {"f64": 1376, "f32": 688, "f16": 344}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_launches(fn, n, stream=None):
    """Average duration of n launches of fn, bracketed by HIP events on the stream the
    library launches on (torch's current stream)."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(n):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / n


def cpu_baseline(su3_small_dims=(8, 32, 32, 32)):
    """The FP64 oracle's D on a bounded sample: an 8 x 32^3 slab (1/8 of the volume) of
    the same field recipe, 3 applications, clover build excluded."""
    import oracle
    from paper_2202_07388_amd import synthetic as syn
    dims = su3_small_dims
    su3, th = syn.gauge_field(dims, EPS, EPS_U1, SEED)
    op = oracle.Operator(dims, su3, th, M0, CSW, -1)
    psi = syn.gaussian_spinor(dims, SEED + 1000)
    op.dw(psi)
    n = 3
    t0 = time.perf_counter()
    for _ in range(n):
        op.dw(psi)
    dt = (time.perf_counter() - t0) / n
    V = int(np.prod(dims))
    return {"value": round(BYTES_PER_SITE["f64"] * V / dt / 1e9, 3), "unit": "GB/s",
            "cores": 1, "kind": "oracle",
            "sample": "oracle D (FP64, single thread) on an 8x32^3 slab of the same "
                      "recipe, mean of 3 applies, clover build excluded; %.3f s per apply"
                      % dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solves", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2202_07388_amd import qdw
    from paper_2202_07388_amd import synthetic as syn

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    qdw.load()
    log("generating 32^3x64 gauge field ...")
    t0 = time.time()
    su3, th = syn.gauge_field(DIMS, EPS, EPS_U1, SEED)
    psi = syn.gaussian_spinor(DIMS, SEED + 1000)
    log("  %.1f s; creating operator" % (time.time() - t0))
    op = qdw.Op(DIMS, su3, th, M0, CSW, -1)
    del su3, th
    V = op.V
    fields = {}
    for prec in ("f64", "f32", "f16"):
        x = op.pack(psi, prec)
        y = op.new_field(prec)
        fields[prec] = (x, y)
    torch.cuda.synchronize()

    x64, y64 = fields["f64"]
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

    extra = {}
    for prec in ("f32", "f16"):
        x, y = fields[prec]
        f = lambda: qdw.dw_apply(op, x, y, prec)
        for _ in range(10):
            f()
        d = time_launches(f, 100)
        extra[prec] = {"ms": round(d * 1e3, 4),
                       "GB_s": round(BYTES_PER_SITE[prec] * V / d / 1e9, 1),
                       "frac_hbm_peak": round(BYTES_PER_SITE[prec] * V / d / 1e9 / HBM_PEAK_GBS, 4)}
    dag = lambda: qdw.dw_dag_apply(op, x64, y64, "f64")
    d_dag = time_launches(dag, 50)
    extra["f64_dag"] = {"ms": round(d_dag * 1e3, 4),
                        "GB_s": round(BYTES_PER_SITE["f64"] * V / d_dag / 1e9, 1)}

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
        "config": {"workload": "Wilson-clover D, 32^3x64, FP64, 12+1-real links",
                   "lattice": "32^3x64", "m0": M0, "c_sw": CSW, "eps": EPS,
                   "eps_u1": EPS_U1, "bc_t": "antiperiodic"},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None},
        "dw_other_precisions": extra,
        "wall_s_timed_region": round(wall, 4),
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on the host (bounded sample) ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
