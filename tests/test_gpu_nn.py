"""The learned gauge-covariant preconditioner through the C ABI against the FP64 oracle.

Tolerances. FP32 mixing (FP32 matrix-core operands, FP32 transport): every product and
sum is rounded at most a few hundred times in binary32 (u = 6e-8) -> 1e-5 relative for
outputs and gradients. bf16 mixing: both GEMM operands are rounded to bf16 (u = 2^-9 =
2e-3) before FP32 accumulation; errors of the K = 576 terms are independent, so the
relative error of an output stays near u: 1e-2 is required.
"""
import numpy as np
import pytest

import oracle
from paper_2202_07388_amd import qdw
from paper_2202_07388_amd import synthetic as syn
from gpu_util import make_pair, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[(4, 4, 4, 4), (6, 4, 4, 6)])
def net(request):
    dims = request.param
    gop, oop, su3, th = make_pair(dims, -0.05, 1.7, 0.3, seed=31)
    W = oracle.nn_identity_weights(seed=3, scale=0.3)
    r = syn.gaussian_spinor(dims, 32)
    return dims, gop, oop, W, r


@pytest.mark.parametrize("f32,tol", [(True, 1e-5), (False, 1e-2)])
def test_forward_matches_oracle(net, f32, tol):
    dims, gop, oop, W, r = net
    w = qdw.nn_weights_tensor(W)
    x = gop.pack(r)
    y = gop.new_field()
    qdw.nn_forward(gop, w, x, y, f32_mixing=f32)
    got = gop.unpack(y).cpu().numpy()
    want, _ = oracle.nn_forward(oop, W, r)
    assert rel(got, want) <= tol, rel(got, want)


def test_identity_weights_are_identity(net):
    dims, gop, oop, W, r = net
    w = qdw.nn_weights_tensor(oracle.nn_identity_weights())
    x = gop.pack(r)
    y = gop.new_field()
    qdw.nn_forward(gop, w, x, y, f32_mixing=True)
    got = gop.unpack(y).cpu().numpy()
    want = r.real.astype(np.float32) + 1j * r.imag.astype(np.float32)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("f32,tol", [(True, 1e-4), (False, 3e-2)])
def test_backward_matches_oracle(net, f32, tol):
    dims, gop, oop, W, r = net
    e = syn.gaussian_spinor(dims, 33)
    L, g, acts = oracle.nn_loss(oop, W, r, e)
    grads, gin = oracle.nn_backward(oop, W, acts, g)
    w = qdw.nn_weights_tensor(W)
    import torch
    dW = torch.zeros_like(w)
    gi = gop.new_field()
    qdw.nn_backward(gop, w, gop.pack(r), gop.pack(2.0 * g), dW, gi, f32_mixing=f32)
    got_w = qdw.nn_weights_layers(dW)
    for l in range(3):
        assert rel(got_w[l], grads[l]) <= tol, (l, rel(got_w[l], grads[l]))
    assert rel(gop.unpack(gi).cpu().numpy(), 2.0 * gin) <= tol


def test_gradients_finite_differences_on_gpu(net):
    """Central differences of the GPU forward (FP32 mixing) against the GPU backward. The
    loss is exactly quadratic in any single weight (the network is linear in each layer's
    weights), so a large step h is exact and keeps FP32 cancellation small."""
    dims, gop, oop, W, r = net
    import torch
    e = syn.gaussian_spinor(dims, 34)
    x = gop.pack(r)
    y = gop.new_field()
    ne2 = np.vdot(e, e).real

    def loss(wt):
        qdw.nn_forward(gop, wt, x, y, f32_mixing=True)
        d = gop.unpack(y).cpu().numpy() - e
        return np.vdot(d, d).real / ne2

    w = qdw.nn_weights_tensor(W)
    qdw.nn_forward(gop, w, x, y, f32_mixing=True)
    g = 2.0 * (gop.unpack(y).cpu().numpy() - e) / ne2
    dW = torch.zeros_like(w)
    gi = gop.new_field()
    qdw.nn_backward(gop, w, x, gop.pack(g), dW, gi, f32_mixing=True)
    dw = dW.cpu().numpy()
    rng = np.random.default_rng(5)
    h = 0.5
    for idx in rng.choice(w.numel(), 12, replace=False):
        wp, wm = w.clone(), w.clone()
        wp[idx] += h
        wm[idx] -= h
        fd = (loss(wp) - loss(wm)) / (2 * h)
        assert abs(fd - dw[idx]) <= 2e-3 * max(1.0, abs(dw[idx])) + 1e-5, (idx, fd, dw[idx])


def test_gauge_equivariance_on_gpu():
    dims = (4, 4, 4, 4)
    su3, th = syn.gauge_field(dims, 0.3, 0.1, 41)
    G = syn.random_gauge_transform(dims, 42)
    nb = oracle.neighbours(dims)
    u = oracle.u3_links(su3, th)
    ug = np.einsum("xij,xmjk,xmlk->xmil", G, u, np.conj(G[nb[:, 0::2]]))
    thg = np.angle(np.linalg.det(ug)) / 3.0
    su3g = ug * np.exp(-1j * thg)[..., None, None]
    a = qdw.Op(dims, su3, th, -0.05, 1.7)
    b = qdw.Op(dims, su3g, thg, -0.05, 1.7)
    W = qdw.nn_weights_tensor(oracle.nn_identity_weights(seed=4, scale=0.3))
    r = syn.gaussian_spinor(dims, 43)
    ya, yb = a.new_field(), b.new_field()
    qdw.nn_forward(a, W, a.pack(r), ya, f32_mixing=True)
    qdw.nn_forward(b, W, b.pack(np.einsum("xij,xsj->xsi", G, r)), yb, f32_mixing=True)
    lhs = b.unpack(yb).cpu().numpy()
    rhs = np.einsum("xij,xsj->xsi", G, a.unpack(ya).cpu().numpy())
    assert rel(lhs, rhs) <= 1e-5


def test_training_reduces_loss():
    """A few Adam steps on solver-style pairs (e = D^-1 r) lower the loss."""
    import torch
    dims = (8, 4, 4, 8)
    gop, oop, _, _ = make_pair(dims, -0.05, 1.7, 0.3, seed=51)
    pairs = []
    for k in range(4):
        e = syn.gaussian_spinor(dims, 60 + k)
        r = oop.dw(e)
        pairs.append((gop.pack(r), gop.pack(e)))
    w = qdw.nn_weights_tensor(oracle.nn_identity_weights(seed=7, scale=0.01))
    adam = torch.zeros(4 * qdw.nn_weight_count(), dtype=torch.float32, device=w.device)
    losses = [qdw.nn_train_step(gop, w, adam, s + 1, 1e-2, [p[0] for p in pairs],
                                [p[1] for p in pairs]) for s in range(60)]
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.7 * losses[0], losses[::10]


@pytest.fixture(scope="module")
def trained():
    """Solver-generated pairs on an 8^4 lattice, a short GPU training run."""
    from paper_2202_07388_amd import nn_train
    dims = (8, 8, 8, 8)
    gop, oop, _, _ = make_pair(dims, -0.05, 1.7, 0.3, seed=7388 + 40)
    etas = [gop.pack(syn.gaussian_spinor(dims, 7388 + 40 + 1000 + k)) for k in range(4)]
    rhos, errs = nn_train.solver_pairs(gop, etas, 24, store="bf16")
    w, losses = nn_train.train(gop, rhos, errs, "bf16", epochs=6, batch=8, lr=5e-3, m0=-0.05)
    return dims, gop, oop, w, losses, len(rhos)


def test_solver_pairs_are_residual_error_pairs():
    """e_k = D^-1 rho_k for the generated pairs (checked with the oracle)."""
    from paper_2202_07388_amd import nn_train
    dims = (4, 4, 4, 8)
    gop, oop, _, _ = make_pair(dims, -0.05, 1.7, 0.3, seed=3)
    eta = gop.pack(syn.gaussian_spinor(dims, 4))
    rhos, errs = nn_train.solver_pairs(gop, [eta], 5, store="f64")
    assert len(rhos) == 5
    for r, e in zip(rhos, errs):
        rn, en = gop.unpack(r).cpu().numpy(), gop.unpack(e).cpu().numpy()
        assert rel(oop.dw(en), rn) <= 1e-10


def test_training_lowers_loss_and_preconditions(trained):
    dims, gop, oop, w, losses, npairs = trained
    assert npairs >= 80 and np.isfinite(losses).all()
    k = max(1, len(losses) // 6)
    assert np.mean(losses[-k:]) < 0.9 * np.mean(losses[:k]), (losses[:k], losses[-k:])
    eta = gop.pack(syn.gaussian_spinor(dims, 99))
    x0, x1 = gop.new_field(), gop.new_field()
    plain = qdw.sap_gcr_solve(gop, eta, x0, res=1e-10, precond="none")
    learned = qdw.sap_gcr_solve(gop, eta, x1, res=1e-10, precond="nn", nn_weights=w)
    assert learned["status"] > 0 and learned["rel_res_true"] <= 1e-10
    # what the trained network gains over GCR without it
    assert learned["status"] < 0.8 * plain["status"], (learned, plain)
    xo, st = oracle.fgcr(oop, syn.gaussian_spinor(dims, 99), 1e-11, 3000, 16)
    assert rel(gop.unpack(x1).cpu().numpy(), xo) <= 1e-7


def test_bad_network_falls_back_to_sap(trained):
    """With QDW_PRECOND_NN_SAP a useless network hands the solve over to SAP."""
    dims, gop, oop, w, losses, npairs = trained
    import torch
    bad = torch.zeros_like(w)
    eta = gop.pack(syn.gaussian_spinor(dims, 98))
    x = gop.new_field()
    info = qdw.sap_gcr_solve(gop, eta, x, res=1e-10, precond="nn_sap", nn_weights=bad,
                             ncy=5, nmr=4, sdtype="f16")
    assert info["status"] > 0 and info["rel_res_true"] <= 1e-10
    assert info["n_dw_lo"] > 0  # SAP did the work


def _dirac_weights(m0):
    """Layer 2 multiplies by D at c_sw = 0 (W_0 = (4 + m0), W_{+-mu} = -1/2 (1 -+ gamma_mu)),
    routed through channels 3 and 5; layers 1 and 3 copy (the oracle test of the same
    weights pins them against oracle.c's operator)."""
    g = oracle.gamma()
    W1 = np.zeros((9, 8, 1, 4, 4), dtype=np.complex128)
    W2 = np.zeros((9, 8, 8, 4, 4), dtype=np.complex128)
    W3 = np.zeros((9, 1, 8, 4, 4), dtype=np.complex128)
    W1[0, 3, 0] = np.eye(4)
    W2[0, 5, 3] = (4.0 + m0) * np.eye(4)
    for mu in range(4):
        W2[1 + 2 * mu, 5, 3] = -0.5 * (np.eye(4) - g[mu])
        W2[2 + 2 * mu, 5, 3] = -0.5 * (np.eye(4) + g[mu])
    W3[0, 0, 5] = np.eye(4)
    return [W1, W2, W3]


@pytest.mark.parametrize("dims", [(6, 4, 4, 6), (16, 8, 8, 8)])
@pytest.mark.parametrize("f32,tol", [(True, 1e-5), (False, 1e-2)])
def test_dirac_weights_give_the_operator(dims, f32, tol):
    """Through the C ABI, the network with Dirac weights equals the oracle's D at c_sw = 0
    (m0 = -0.5, so every weight is exact in bf16): the GPU's spin, channel and path
    conventions are those of the operator itself."""
    gop, oop, _, _ = make_pair(dims, -0.5, 0.0, 0.3, seed=35)
    r = syn.gaussian_spinor(dims, 36)
    y = gop.new_field()
    qdw.nn_forward(gop, qdw.nn_weights_tensor(_dirac_weights(-0.5)), gop.pack(r), y,
                   f32_mixing=f32)
    got = gop.unpack(y).cpu().numpy()
    want = oop.dw(r)
    assert rel(got, want) <= tol, rel(got, want)
    gop.close()


@pytest.fixture(scope="module")
def net16():
    """16 x 8^3 (8192 sites, several 64-site tiles per time slice) with random weights: the
    oracle's forward pass, loss gradient and backward pass, computed once."""
    dims = (16, 8, 8, 8)
    gop, oop, _, _ = make_pair(dims, -0.05, 1.7, 0.3, seed=37)
    W = oracle.nn_identity_weights(seed=8, scale=0.3)
    r = syn.gaussian_spinor(dims, 38)
    e = syn.gaussian_spinor(dims, 39)
    out, _ = oracle.nn_forward(oop, W, r)
    L, g, acts = oracle.nn_loss(oop, W, r, e)
    grads, gin = oracle.nn_backward(oop, W, acts, g)
    yield gop, W, r, out, g, grads, gin
    gop.close()


@pytest.mark.parametrize("f32,tol,gtol", [(True, 1e-5, 1e-4), (False, 1e-2, 3e-2)])
def test_random_weights_16x8c3(net16, f32, tol, gtol):
    import torch
    gop, W, r, out, g, grads, gin = net16
    w = qdw.nn_weights_tensor(W)
    y = gop.new_field()
    qdw.nn_forward(gop, w, gop.pack(r), y, f32_mixing=f32)
    assert rel(gop.unpack(y).cpu().numpy(), out) <= tol
    dW = torch.zeros_like(w)
    gi = gop.new_field()
    qdw.nn_backward(gop, w, gop.pack(r), gop.pack(2.0 * g), dW, gi, f32_mixing=f32)
    got_w = qdw.nn_weights_layers(dW)
    for l in range(3):
        assert rel(got_w[l], grads[l]) <= gtol, (l, rel(got_w[l], grads[l]))
    assert rel(gop.unpack(gi).cpu().numpy(), 2.0 * gin) <= gtol


@pytest.mark.parametrize("kind", ["error", "dnorm"])
def test_train_step_loss_and_first_adam_step(kind):
    """One training step against the oracle: the returned batch loss (before the update)
    is the mean over the pairs of |N(r) - e|^2 / |e|^2 ("error") or |D(N(r) - e)|^2 /
    |D e|^2 ("dnorm") with the oracle's network and operator, within the bf16 mixing's
    error; and the first Adam step from a zero state moves every weight by lr against the
    sign of its gradient (bias-corrected m / sqrt(v) = g / |g| at step 1), checked on the
    components whose oracle gradient is large enough for the bf16 gradient's sign to be
    certain."""
    import torch
    dims = (4, 4, 4, 4)
    gop, oop, _, _ = make_pair(dims, -0.05, 1.7, 0.3, seed=71)
    W = oracle.nn_identity_weights(seed=5, scale=0.3)
    rs = [syn.gaussian_spinor(dims, 72 + k) for k in range(2)]
    es = [syn.gaussian_spinor(dims, 82 + k) for k in range(2)]
    want, grad = 0.0, None
    for r, e in zip(rs, es):
        out, acts = oracle.nn_forward(oop, W, r)
        d = out - e
        if kind == "error":
            den = np.vdot(e, e).real
            L, g = np.vdot(d, d).real / den, d / den
        else:
            Dd, De = oop.dw(d), oop.dw(e)
            den = np.vdot(De, De).real
            L, g = np.vdot(Dd, Dd).real / den, oop.dw_dag(Dd) / den
        want += L / len(rs)
        gl, _ = oracle.nn_backward(oop, W, acts, g)
        grad = gl if grad is None else [a + b for a, b in zip(grad, gl)]
    w = qdw.nn_weights_tensor(W)
    w0 = w.detach().cpu().numpy().copy()
    adam = torch.zeros(4 * qdw.nn_weight_count(), dtype=torch.float32, device=w.device)
    lr = 1e-2
    got = qdw.nn_train_step(gop, w, adam, 1, lr, [gop.pack(r) for r in rs],
                            [gop.pack(e) for e in es], "f64", kind)
    assert abs(got - want) <= 5e-2 * want, (got, want)
    delta = w.detach().cpu().numpy().astype(np.float64) - w0
    gflat = np.concatenate([x.reshape(-1) for x in grad])
    gri = np.stack([gflat.real, gflat.imag], axis=-1).reshape(-1)
    sure = np.abs(gri) > 0.05 * np.abs(gri).max()
    assert sure.sum() >= 100
    assert np.abs(delta[sure] + lr * np.sign(gri[sure])).max() <= 1e-3 * lr
    assert np.abs(delta).max() <= lr * (1 + 1e-3)
