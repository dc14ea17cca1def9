"""Training pipeline of the learned preconditioner (library calls only).

Pairs come from the solver itself: for a source eta, the iterates psi_k of plain FP64
flexible GCR after k = 1, 2, ... steps give the residual rho_k = eta - D psi_k and the
error e_k = x* - psi_k = D^-1 rho_k, with x* the solution to 1e-12. The network is then
fitted to rho_k -> e_k by Adam on the GPU (nn_train_step: forward, loss, backward and
update all in the library's kernels), with the error measured in the D-norm by default.
"""
from __future__ import annotations

import numpy as np

from . import qdw


def init_weights(m0: float, seed: int, noise: float = 1e-3):
    """Start from N(r) = r / (4 + m0) (the inverse of the operator's diagonal in the free
    field): the identity path of each layer carries (4 + m0)^(-1/3) on channel 0, plus
    small complex noise everywhere so that all channels can learn."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = (4.0 + m0) ** (-1.0 / 3.0)
    layers = []
    for cin, cout in zip(qdw.NN_CHANNELS[:-1], qdw.NN_CHANNELS[1:]):
        shape = (qdw.NN_PATHS, cout, cin, 4, 4)
        W = noise * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
        W[0, 0, 0] += c * np.eye(4)
        layers.append(W)
    return layers


def solver_pairs(op: "qdw.Op", etas, steps: int, store: str = "bf16", nkv: int = 16,
                 log=None):
    """Residual/error pairs from plain FP64 GCR (restart nkv) on the given FP64 sources.

    The iterate after m full cycles and j more steps is psi_{m nkv} plus the iterate of a
    GCR run of j steps from zero on the residual eta - D psi_{m nkv} (a restart is exactly
    such a fresh start), so the pairs of one cycle come from runs of 1..nkv steps on that
    cycle's residual: sum_j j = nkv (nkv + 1) / 2 applications of D per cycle, instead of
    rerunning the whole solve from zero for every k."""
    rhos, errs = [], []
    xs = op.new_field("f64")
    delta = op.new_field("f64")
    base = op.new_field("f64")
    src = op.new_field("f64")
    psi = op.new_field("f64")
    t = op.new_field("f64")

    def keep(rho, err):
        if store == "f64":
            rhos.append(rho)
            errs.append(err)
            return
        r_s, e_s = op.new_field(store), op.new_field(store)
        n2 = qdw.norm2(op, rho)
        s = np.sqrt(24.0 * op.V / n2)           # unit component size for storage
        qdw.convert(op, rho, "f64", r_s, store, s)
        qdw.convert(op, err, "f64", e_s, store, s)
        rhos.append(r_s)
        errs.append(e_s)

    for n, eta in enumerate(etas):
        info = qdw.sap_gcr_solve(op, eta, xs, res=1e-12, nmx=20000, nkv=nkv, precond="none")
        if info["status"] <= 0:
            raise qdw.QdwError("pair generation: reference solve failed: %s" % info)
        qdw.axpby(op, 0.0, eta, 0.0, base)           # psi_0 = 0
        qdw.axpby(op, 1.0, eta, 0.0, src)            # its residual
        k, done = 0, False
        while k < steps and not done:
            for j in range(1, nkv + 1):
                inf = qdw.sap_gcr_solve(op, src, delta, res=1e-14, nmx=j, nkv=nkv,
                                        precond="none")
                qdw.axpby(op, 1.0, base, 0.0, psi)
                qdw.axpby(op, 1.0, delta, 1.0, psi)  # psi_k = psi_base + delta
                if inf["status"] >= 0:
                    done = True                     # converged: no further useful pairs
                    break
                qdw.dw_apply(op, psi, t, "f64")
                rho = op.new_field("f64")
                qdw.axpby(op, 1.0, eta, 0.0, rho)
                qdw.axpby(op, -1.0, t, 1.0, rho)      # rho = eta - D psi
                err = op.new_field("f64")
                qdw.axpby(op, 1.0, xs, 0.0, err)
                qdw.axpby(op, -1.0, psi, 1.0, err)    # e = x* - psi
                keep(rho, err)
                del rho, err
                k += 1
                if k >= steps:
                    break
            # next cycle: from the iterate after nkv steps
            qdw.axpby(op, 1.0, psi, 0.0, base)
            qdw.dw_apply(op, base, t, "f64")
            qdw.axpby(op, 1.0, eta, 0.0, src)
            qdw.axpby(op, -1.0, t, 1.0, src)
        if log:
            log("pairs: source %d done, %d pairs" % (n, len(rhos)))
    return rhos, errs


def train(op: "qdw.Op", rhos, errs, store: str, epochs: int, batch: int, lr: float,
          m0: float, seed: int = 0, loss: str = "dnorm", log=None, groups=None):
    """Adam on the pairs; returns the weights tensor and the loss per step. The default
    loss measures N(rho) - e in the D-norm, i.e. the residual a GCR step would leave,
    which is what the flexible GCR judges a preconditioner by.

    Pairs from several gauge fields: pass groups = [(op_f, rhos_f, errs_f), ...] (op, rhos
    and errs are then ignored); every batch is drawn from one field, since the network's
    transports and the loss's D use that field's links."""
    import torch
    if groups is None:
        groups = [(op, rhos, errs)]
    w = qdw.nn_weights_tensor(init_weights(m0, seed))
    adam = torch.zeros(4 * qdw.nn_weight_count(), dtype=torch.float32, device=w.device)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    losses = []
    step = 0
    for ep in range(epochs):
        batches = []
        for gi, (_, rs, _) in enumerate(groups):
            order = rng.permutation(len(rs))
            batches += [(gi, order[b0:b0 + batch]) for b0 in range(0, len(order) - batch + 1, batch)]
        nb = len(batches)
        for j in rng.permutation(nb):
            gi, idx = batches[j]
            gop, rs, es = groups[gi]
            step += 1
            losses.append(qdw.nn_train_step(gop, w, adam, step, lr, [rs[i] for i in idx],
                                            [es[i] for i in idx], store, loss))
        if log:
            log("epoch %d: mean loss %.4f" % (ep, float(np.mean(losses[-max(1, nb):]))))
    return w, losses


STATE_FORMAT = "qdw-nn-1-8-8-1"


def save_state(path: str, weights, adam=None, step: int = 0, meta=None) -> None:
    """Write the network's weights (the library's FP32 interleaved layout) and, to resume
    training, the Adam moments and step count to a safetensors file (tensors and string
    metadata only: loading it runs no code from the file)."""
    from safetensors.torch import save_file
    tensors = {"weights": weights.detach().to("cpu").contiguous()}
    if adam is not None:
        tensors["adam"] = adam.detach().to("cpu").contiguous()
    md = {"format": STATE_FORMAT, "step": str(int(step))}
    md.update({str(k): str(v) for k, v in (meta or {}).items()})
    save_file(tensors, path, metadata=md)


def load_state(path: str, device=None):
    """Read what save_state wrote: (weights, adam or None, step, metadata), the tensors on
    `device` (CPU if None). Refuses a file of another format or with tensors of the wrong
    size for the 1-8-8-1 network."""
    from safetensors import safe_open
    with safe_open(path, framework="pt", device="cpu") as f:
        md = dict(f.metadata() or {})
        if md.get("format") != STATE_FORMAT:
            raise ValueError("%s: not a network state file (format %r)" % (path, md.get("format")))
        keys = set(f.keys())
        w = f.get_tensor("weights")
        adam = f.get_tensor("adam") if "adam" in keys else None
    n = qdw.nn_weight_count()
    if w.numel() != 2 * n or (adam is not None and adam.numel() != 4 * n):
        raise ValueError("%s: tensor sizes do not match the 1-8-8-1 network" % path)
    if device is not None:
        w = w.to(device)
        adam = adam.to(device) if adam is not None else None
    return w, adam, int(md.get("step", "0")), md


def _time_forward(dims, reps: int = 5):
    """Time the network's forward pass (bf16 matrix-core mixing) on a random field of the
    given extents, with the identity-path initial weights plus noise."""
    import time
    import torch
    from . import synthetic as syn
    su3, th = syn.gauge_field(dims, 0.3, 0.1, 7388)
    op = qdw.Op(dims, su3, th, -0.05, 1.7)
    del su3, th
    w = qdw.nn_weights_tensor(init_weights(-0.05, 0, noise=0.1))
    x = op.pack(syn.gaussian_spinor(dims, 3))
    y = op.new_field()
    qdw.nn_forward(op, w, x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        qdw.nn_forward(op, w, x, y)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    print("nn_forward %s: %.3f ms per application" % ("x".join(map(str, dims)), ms), flush=True)
    op.close()


if __name__ == "__main__":
    import sys
    _time_forward(tuple(int(v) for v in (sys.argv[1] if len(sys.argv) > 1 else "64,32,32,32").split(",")))
