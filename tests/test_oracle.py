"""Pins of the FP64 CPU oracle against facts fixed by mathematics and the paper.

None of these re-types an oracle formula: each check goes through an independent
route (closed forms, brute-force dense matrices, algebraic identities, optimality
properties of the Krylov methods) chosen so that a dropped term, a wrong sign or index,
or a transposed operand in the oracle fails at least one of them.
"""
import numpy as np
import pytest

import oracle
from paper_2202_07388_amd import synthetic as syn

D44 = (4, 4, 4, 4)


def _op(dims, m0=0.1, csw=1.5, eps=0.3, seed=7388, bc=-1):
    su3, th = syn.gauge_field(dims, eps, 0.1, seed)
    return oracle.Operator(dims, su3, th, m0, csw, bc)


@pytest.fixture(scope="module")
def op44():
    return _op(D44)


@pytest.fixture(scope="module")
def dense44(op44):
    return oracle.dense_matrix(op44)


def spin(m, v):
    return np.einsum("st,xtc->xsc", m, v)


# ----------------------------------------------------------------- basis, geometry

def test_gamma_clifford_and_chiral_basis():
    g = oracle.gamma()
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T)
        for n in range(4):
            assert np.allclose(g[m] @ g[n] + g[n] @ g[m], 2.0 * (m == n) * np.eye(4))
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))
    # every sigma_{mu nu} is block diagonal in this basis (chirality is conserved)
    for m in range(4):
        for n in range(4):
            s = 0.5j * (g[m] @ g[n] - g[n] @ g[m])
            assert np.allclose(s[:2, 2:], 0) and np.allclose(s[2:, :2], 0)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 2, 4, 8)])
def test_neighbours_round_trip(dims):
    nb = oracle.neighbours(dims)
    V = int(np.prod(dims))
    idx = np.arange(V)
    x = np.indices(dims).reshape(4, -1)
    for mu in range(4):
        f, b = nb[:, 2 * mu], nb[:, 2 * mu + 1]
        assert np.array_equal(nb[f, 2 * mu + 1], idx)
        assert np.array_equal(nb[b, 2 * mu], idx)
        y = x.copy()
        y[mu] = (y[mu] + 1) % dims[mu]
        lex = ((y[0] * dims[1] + y[1]) * dims[2] + y[2]) * dims[3] + y[3]
        assert np.array_equal(f, lex)
    par = x.sum(axis=0) % 2
    assert (par == 0).sum() == V // 2


def test_generator_links_in_su3_times_u1():
    su3, th = syn.gauge_field(D44, 0.3, 0.1, 1)
    u = su3.reshape(-1, 3, 3)
    err = np.abs(u @ np.conj(np.swapaxes(u, 1, 2)) - np.eye(3)).max()
    assert err < 1e-14
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-14
    # the third row is exactly what a compressed two-row link rebuilds
    assert np.abs(u[:, 2] - np.conj(np.cross(u[:, 0], u[:, 1]))).max() < 1e-15
    full = oracle.u3_links(su3, th).reshape(-1, 3, 3)
    assert np.allclose(np.linalg.det(full), np.exp(3j * th.reshape(-1)))


# ----------------------------------------------------------------- free field

@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (16, 8, 8, 8)])
def test_free_field_plane_waves(dims):
    """D e^{ipx} u = [m0 + sum(1 - cos p) + i sum gamma sin p] e^{ipx} u, with
    antiperiodic time momenta p0 = pi(2n+1)/T and periodic p_k = 2 pi n / L_k."""
    su3, th = syn.unit_gauge_field(dims)
    m0 = 0.1
    op = oracle.Operator(dims, su3, th, m0, 1.5, -1)
    g = oracle.gamma()
    rng = np.random.default_rng(3)
    for _ in range(4):
        n = [rng.integers(0, d) for d in dims]
        p = np.array([np.pi * (2 * n[0] + 1) / dims[0]] +
                     [2 * np.pi * n[k] / dims[k] for k in (1, 2, 3)])
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = syn.plane_wave(dims, p, u)
        Dp = (m0 + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(
            g[m] * np.sin(p[m]) for m in range(4))
        got = op.dw(psi)
        assert np.abs(got - spin(Dp, psi)).max() < 1e-13 * np.abs(psi).max()
        got_d = op.dw_dag(psi)
        assert np.abs(got_d - spin(Dp.conj().T, psi)).max() < 1e-13 * np.abs(psi).max()


def test_periodic_time_plane_wave():
    """With bc_t = +1 the time momenta are 2 pi n / T instead."""
    dims = (4, 4, 4, 4)
    su3, th = syn.unit_gauge_field(dims)
    op = oracle.Operator(dims, su3, th, -0.3, 1.0, +1)
    g = oracle.gamma()
    p = np.array([2 * np.pi / 4, 0, 2 * np.pi * 3 / 4, 2 * np.pi / 4])
    u = np.arange(12).reshape(4, 3) + 0.5j
    psi = syn.plane_wave(dims, p, u)
    Dp = (-0.3 + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(
        g[m] * np.sin(p[m]) for m in range(4))
    assert np.abs(op.dw(psi) - spin(Dp, psi)).max() < 1e-13 * np.abs(psi).max()


# ----------------------------------------------------------------- gamma5, gauge

@pytest.mark.parametrize("dims, bc", [((4, 4, 4, 4), -1), ((6, 4, 4, 6), 1), ((6, 4, 4, 6), -1)])
def test_dw_at_sites_equals_full_operator(dims, bc):
    """The per-site evaluation used to sample large lattices (its own stencil and clover
    code) agrees with the full operator at every site."""
    su3, th = syn.gauge_field(dims, 0.3, 0.1, 7388 + dims[0])
    op = oracle.Operator(dims, su3, th, -0.05, 1.7, bc)
    psi = syn.gaussian_spinor(dims, 50)
    want = op.dw(psi)
    sites = np.arange(op.V)
    got = oracle.dw_at_sites(dims, bc, op.u, -0.05, 1.7, psi, sites)
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()
    # and on a scattered subset, in a scrambled order
    sub = np.random.default_rng(1).permutation(op.V)[:37]
    got = oracle.dw_at_sites(dims, bc, op.u, -0.05, 1.7, psi, sub)
    assert np.abs(got - want[sub]).max() <= 1e-14 * np.abs(want).max()


def test_gamma5_hermiticity(op44):
    x = syn.gaussian_spinor(D44, 11)
    y = syn.gaussian_spinor(D44, 12)
    g5 = np.diag([1.0, 1.0, -1.0, -1.0])
    lhs = np.vdot(y, op44.dw(x))
    rhs = np.vdot(op44.dw_dag(y), x)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    g5dg5 = spin(g5, op44.dw(spin(g5, x)))
    assert np.abs(g5dg5 - op44.dw_dag(x)).max() < 1e-14 * np.abs(x).max()


def test_gauge_covariance():
    dims = (4, 4, 2, 6)
    su3, th = syn.gauge_field(dims, 0.3, 0.1, 5)
    G = syn.random_gauge_transform(dims, 6)
    op = oracle.Operator(dims, su3, th, 0.2, 1.3, -1)
    u = op.u
    nb = oracle.neighbours(dims)
    # U^g_mu(x) = G(x) U_mu(x) G(x + mu)^+ , split back into SU(3) x U(1)
    ug = np.einsum("xij,xmjk,xmlk->xmil", G, u, np.conj(G[nb[:, 0::2]]))
    det = np.linalg.det(ug)
    thg = np.angle(det) / 3.0
    su3g = ug * np.exp(-1j * thg)[..., None, None]
    opg = oracle.Operator(dims, su3g, thg, 0.2, 1.3, -1)
    assert np.abs(opg.u - ug).max() < 1e-13
    psi = syn.gaussian_spinor(dims, 7)
    Gpsi = np.einsum("xij,xsj->xsi", G, psi)
    lhs = opg.dw(Gpsi)
    rhs = np.einsum("xij,xsj->xsi", G, op.dw(psi))
    assert np.abs(lhs - rhs).max() < 1e-13 * np.abs(rhs).max()
    # clover term transforms as A -> G A G^+ (G acting on colour)
    Gs = np.einsum("st,xij->xsitj", np.eye(4), G).reshape(-1, 12, 12)
    assert np.abs(opg.A - Gs @ op.A @ np.conj(np.swapaxes(Gs, 1, 2))).max() < 1e-13


# ----------------------------------------------------------------- clover term

def test_clover_hermitian_chiral_trace(op44):
    A = op44.A
    assert np.abs(A - np.conj(np.swapaxes(A, 1, 2))).max() < 1e-14
    assert np.abs(A[:, :6, 6:]).max() == 0 and np.abs(A[:, 6:, :6]).max() == 0
    # sigma_{mu nu} is traceless within each chirality: tr A_+- = 6 (4 + m0)
    tr_p = np.trace(A[:, :6, :6], axis1=1, axis2=2)
    tr_m = np.trace(A[:, 6:, 6:], axis1=1, axis2=2)
    assert np.abs(tr_p - 6 * 4.1).max() < 1e-13
    assert np.abs(tr_m - 6 * 4.1).max() < 1e-13
    # and it is not trivial on this rough field
    assert np.abs(A - 4.1 * np.eye(12)).max() > 0.1


@pytest.mark.parametrize("csw, m0", [(1.5, 0.1), (1.7, -0.3)])
def test_clover_chirality_block_structure(csw, m0):
    """In the chiral basis each sigma_{mu nu} acts on the two spins of a chirality as a
    traceless 2x2 matrix, so the colour blocks of the clover term on a chirality's two spins
    sum to 2 (4 + m0) 1: every chirality block is (4 + m0) 1 + [[H, b], [b^+, -H]] with H
    Hermitian, 27 reals instead of 36 (the compact form the D kernels read). Also with rough
    U(3) links, where the field strength is not traceless."""
    dims = (4, 4, 4, 6)
    su3, th = syn.gauge_field(dims, 0.5, 0.3, 3)
    op = oracle.Operator(dims, su3, th, m0, csw, -1)
    A = op.A
    for blk in (0, 6):
        a = A[:, blk:blk + 3, blk:blk + 3]
        d = A[:, blk + 3:blk + 6, blk + 3:blk + 6]
        assert np.abs(a + d - 2.0 * (4.0 + m0) * np.eye(3)).max() < 1e-14
        H = 0.5 * (a - d)
        assert np.abs(H - np.conj(np.swapaxes(H, 1, 2))).max() < 1e-14
        assert np.abs(a - (4.0 + m0) * np.eye(3)).max() > 0.1  # H itself is not small
    assert np.abs(A[:, 0:6, 6:12]).max() == 0.0


def test_clover_unit_field():
    su3, th = syn.unit_gauge_field(D44)
    op = oracle.Operator(D44, su3, th, -0.05, 1.7, -1)
    assert np.abs(op.A - 3.95 * np.eye(12)).max() < 1e-15


@pytest.mark.parametrize("plane,diag", [((1, 2), [1, -1, 1, -1]), ((0, 3), [-1, 1, 1, -1])])
def test_clover_constant_abelian_flux(plane, diag):
    """Constant flux phi in one plane: every leaf is e^{i phi}, Fhat = i sin(phi), and the
    clover term is -(c_sw/2) sin(phi) sigma_{mu nu}: sigma_12 = diag(-1,1,-1,1),
    sigma_03 = diag(1,-1,-1,1) in the chiral basis."""
    dims = (4, 6, 4, 8)
    su3, _ = syn.unit_gauge_field(dims)
    theta, phi = syn.abelian_flux_theta(dims, 1, plane)
    m0, csw = 0.1, 1.7
    op = oracle.Operator(dims, su3, theta, m0, csw, -1)
    want = (4 + m0) * np.eye(12) + 0.5 * csw * np.sin(phi) * np.kron(np.diag(diag), np.eye(3))
    assert np.abs(op.A - want).max() < 1e-14


# ----------------------------------------------------------------- dense 4^4

def test_dense_structure(dense44):
    """54 non-zeros per row (6 clover + 8 hops x 2 spin x 3 colour) of 3072, ~1.8 %
    (the paper quotes about 2 % for its 4^4 operator)."""
    nnz = (np.abs(dense44) > 0).sum(axis=1)
    assert np.all(nnz == 54)
    assert abs(nnz.sum() / dense44.size - 54 / 3072) < 1e-12


def test_dense_adjoint(op44, dense44):
    dag = oracle.dense_matrix(op44, "dag")
    assert np.abs(dag - dense44.conj().T).max() < 1e-15


def test_even_odd_structure(dense44):
    """Even sites couple to odd sites only through hops: the even-even and odd-odd
    blocks hold nothing but the (site-diagonal) clover term."""
    x = np.indices(D44).reshape(4, -1)
    par = np.repeat(x.sum(axis=0) % 2, 12)
    for p in (0, 1):
        blk = dense44[np.ix_(par == p, par == p)]
        n = blk.shape[0] // 12
        sites = blk.reshape(n, 12, n, 12)
        off = sites.copy()
        off[np.arange(n), :, np.arange(n), :] = 0
        assert np.abs(off).max() == 0


def test_spectrum_conjugate_pairs():
    dims = (4, 2, 2, 2)
    op = _op(dims, m0=-0.2, csw=1.5, eps=0.5, seed=9)
    ev = np.linalg.eigvals(oracle.dense_matrix(op))
    ev_c = np.conj(ev)
    d = np.abs(ev[:, None] - ev_c[None, :]).min(axis=1)
    assert d.max() < 1e-10


# ----------------------------------------------------------------- CGNE

def test_cgne_matches_dense_solve(op44, dense44):
    eta = syn.gaussian_spinor(D44, 7388 + 1000)
    x, status, hist = oracle.cgne(op44, eta, 1e-10, 1000, history=True)
    assert status > 0
    xd = np.linalg.solve(dense44.conj().T @ dense44, eta.reshape(-1))
    # true residual of the normal equations and error against the dense solution
    r = eta - op44.normal(x)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(eta)
    assert np.linalg.norm(x.reshape(-1) - xd) <= 1e-7 * np.linalg.norm(xd)
    # successive directions are A-orthogonal (Fig. 1, panel d)
    a = np.abs(np.array(hist["a_orth"]))
    assert a.max() < 1e-8 * np.linalg.norm(eta) ** 2
    # the exact residual follows the recursive one closely in FP64 (no reset needed)
    gap = np.abs(np.array(hist["exact"]) - np.array(hist["recursive"]))
    assert gap.max() < 1e-11


def test_cg_krylov_optimality(op44, dense44):
    """After k steps CG minimises the A-norm of the error over K_k(A, eta), A = D^+ D."""
    eta = syn.gaussian_spinor(D44, 5).reshape(-1)
    A = dense44.conj().T @ dense44
    xs = np.linalg.solve(A, eta)
    Q = np.zeros((eta.size, 0), dtype=np.complex128)
    v = eta / np.linalg.norm(eta)
    for k in range(1, 13):
        Q = np.column_stack([Q, v])
        w = A @ v
        w -= Q @ (Q.conj().T @ w)
        w -= Q @ (Q.conj().T @ w)
        v = w / np.linalg.norm(w)
        xk, st = oracle.cgne(op44, eta, 1e-30, k)
        assert st == -1
        y = np.linalg.solve(Q.conj().T @ A @ Q, Q.conj().T @ eta)
        xopt = Q @ y
        e_cg = xk.reshape(-1) - xs
        e_opt = xopt - xs
        an = lambda e: np.sqrt(np.vdot(e, A @ e).real)
        assert abs(an(e_cg) - an(e_opt)) <= 1e-9 * an(xs)
        assert np.linalg.norm(xk.reshape(-1) - xopt) <= 1e-8 * np.linalg.norm(xs)


# ----------------------------------------------------------------- FGCR

def test_gcr_residuals_equal_gmres(op44, dense44):
    """Unpreconditioned, unrestarted GCR minimises |eta - D y| over K_k(D, eta): its
    residual norms equal GMRES's, obtained here by dense least squares."""
    eta = syn.gaussian_spinor(D44, 21)
    k_max = 12
    _, st, hist = oracle.fgcr(op44, eta, 1e-30, k_max, 64, None, history=True)
    assert st == -1
    b = eta.reshape(-1)
    K = [b]
    for _ in range(k_max - 1):
        K.append(dense44 @ K[-1])
    for k in range(1, k_max + 1):
        B = np.linalg.qr(np.column_stack(K[:k]))[0]
        y = np.linalg.lstsq(dense44 @ B, b, rcond=None)[0]
        gm = np.linalg.norm(b - dense44 @ (B @ y)) / np.linalg.norm(b)
        assert abs(hist[k - 1] - gm) <= 1e-10 * max(gm, 1e-3)
    assert np.all(np.diff(hist) <= 1e-15)


def test_gcr_exact_preconditioner_one_step(op44, dense44):
    eta = syn.gaussian_spinor(D44, 22)
    Dinv = np.linalg.inv(dense44)
    M = lambda v: (Dinv @ v.reshape(-1)).reshape(v.shape)
    psi, st = oracle.fgcr(op44, eta, 1e-10, 5, 4, M)
    assert st == 1
    assert np.linalg.norm(eta - op44.dw(psi)) <= 1e-10 * np.linalg.norm(eta)


def test_gcr_restarts_match_dense_solve(op44, dense44):
    eta = syn.gaussian_spinor(D44, 23)
    psi, st = oracle.fgcr(op44, eta, 1e-10, 500, 8)
    assert st > 8  # needs several restarts
    xd = np.linalg.solve(dense44, eta.reshape(-1))
    assert np.linalg.norm(psi.reshape(-1) - xd) <= 1e-8 * np.linalg.norm(xd)


# ----------------------------------------------------------------- SAP

BS2 = (2, 2, 2, 2)


def test_block_operator_is_masked_dense(op44, dense44):
    """D_b (hops leaving the block dropped) equals P_b D P_b for every block."""
    Db = oracle.dense_block_matrix(op44, BS2)
    bid, col, nblk = oracle.block_ids(D44, BS2)
    b12 = np.repeat(bid, 12)
    same = b12[:, None] == b12[None, :]
    assert np.array_equal(Db, np.where(same, dense44, 0))


def test_mr_step_minimises_block_residual(op44):
    r = syn.gaussian_spinor(D44, 31)
    bid, col, nblk = oracle.block_ids(D44, BS2)
    chi, rb = oracle.mr_blocks(op44, r, BS2, 0, 1)
    for b in np.unique(bid[col == 0])[:6]:
        m = bid == b
        v = op44.dw_blocks(np.where(m[:, None, None], r, 0), BS2)[m].reshape(-1)
        r0 = r[m].reshape(-1)
        # closed form of one MR step: |r1|^2 = |r0|^2 - |v^+ r0|^2 / |v|^2
        want = np.vdot(r0, r0).real - abs(np.vdot(v, r0)) ** 2 / np.vdot(v, v).real
        assert abs(np.vdot(rb[m], rb[m]).real - want) < 1e-12 * np.vdot(r0, r0).real
        # and the block residual is r0 - D_b chi
        res = r0 - op44.dw_blocks(np.where(m[:, None, None], chi, 0), BS2)[m].reshape(-1)
        assert np.abs(res - rb[m].reshape(-1)).max() < 1e-13
    assert np.abs(chi[col == 1]).max() == 0


def test_mr_norm_never_increases(op44):
    r = syn.gaussian_spinor(D44, 32)
    _, _, norms = oracle.mr_blocks(op44, r, BS2, 1, 8, history=True)
    n = np.array(norms)
    bid, col, _ = oracle.block_ids(D44, BS2)
    used = np.unique(bid[col == 1])
    assert np.all(np.diff(n[:, used], axis=0) <= 1e-14)


def test_sap_cycle_is_block_gauss_seidel(op44, dense44):
    """MR iterated to convergence makes one SAP cycle the block Gauss-Seidel sweep
    psi_b = D_bb^-1 rho_b; psi_w = D_ww^-1 (rho - D psi_b)_w."""
    rho = syn.gaussian_spinor(D44, 33)
    bid, col, _ = oracle.block_ids(D44, BS2)
    c12 = np.repeat(col, 12)
    b, w = c12 == 0, c12 == 1
    r = rho.reshape(-1)
    psi = np.zeros_like(r)
    psi[b] = np.linalg.solve(dense44[np.ix_(b, b)], r[b])
    res = r - dense44 @ psi
    psi[w] = np.linalg.solve(dense44[np.ix_(w, w)], res[w])
    got = oracle.sap(op44, rho, BS2, 1, 150).reshape(-1)
    assert np.linalg.norm(got - psi) <= 1e-9 * np.linalg.norm(psi)


def test_sap_zero_cycles_is_identity(op44):
    rho = syn.gaussian_spinor(D44, 34)
    assert np.array_equal(oracle.sap(op44, rho, BS2, 0, 4), rho)


def test_sap_gcr_converges_to_dense_solution(op44, dense44):
    eta = syn.gaussian_spinor(D44, 35)
    M = lambda v: oracle.sap(op44, v, BS2, 3, 4)
    psi, st = oracle.fgcr(op44, eta, 1e-10, 200, 16, M)
    _, st0 = oracle.fgcr(op44, eta, 1e-10, 500, 16, None)
    assert 0 < st < st0
    xd = np.linalg.solve(dense44, eta.reshape(-1))
    assert np.linalg.norm(psi.reshape(-1) - xd) <= 1e-8 * np.linalg.norm(xd)


def test_adaptive_sap_exit_rules(op44):
    rho = syn.gaussian_spinor(D44, 36)
    psi, cycles, steps = oracle.sap_adaptive(op44, rho, BS2, 20, 20, 0.9, 0.0)
    assert 1 <= cycles <= 20
    assert all(np.all((s >= 1) & (s <= 20)) for s in steps)
    r = np.linalg.norm(rho - op44.dw(psi))
    assert r < np.linalg.norm(rho)
    # a huge tolerance makes every block exit at once (rule 3): nothing is done, so the first
    # cycle leaves |r| unchanged and the cycle exit (a cycle that did not lower |r|) fires
    # after exactly one cycle; a strict comparison (|r| grew) would run all 20
    psi0, c0, s0 = oracle.sap_adaptive(op44, rho, BS2, 20, 20, 0.9, 1e30)
    assert c0 == 1 and np.abs(psi0).max() == 0 and all(np.all(s == 0) for s in s0)


def test_adaptive_sap_without_exits_is_plain_sap(op44):
    """With alpha so large that exit (1) never fires and tol = 0, adaptive SAP runs every
    block for nmr_max MR steps in every cycle (MR never raises the block residual, so exit (2)
    stays off) as long as each cycle lowers |r|: it is the plain SAP of Sec. 3, which the
    block Gauss-Seidel pin fixes."""
    rho = syn.gaussian_spinor(D44, 37)
    psi, cycles, steps = oracle.sap_adaptive(op44, rho, BS2, 3, 6, 1e300, 0.0)
    assert cycles == 3 and all(np.all(s == 6) for s in steps)
    want = oracle.sap(op44, rho, BS2, 3, 6)
    assert np.abs(psi - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("nmr_max, expect", [(10, 4), (3, 3)])
def test_adaptive_sap_alpha_zero_stops_after_four_steps(op44, nmr_max, expect):
    """alpha = 0 makes exit (1) fire at the first step it may look at, which Sec. 3.2 puts
    after at least four MR steps: every block takes exactly 4 steps (or nmr_max if smaller),
    so the application equals plain SAP with nmr = 4 (or nmr_max)."""
    rho = syn.gaussian_spinor(D44, 38)
    psi, cycles, steps = oracle.sap_adaptive(op44, rho, BS2, 2, nmr_max, 0.0, 0.0)
    assert cycles == 2 and all(np.all(s == expect) for s in steps)
    want = oracle.sap(op44, rho, BS2, 2, expect)
    assert np.abs(psi - want).max() <= 1e-13 * np.abs(want).max()


def _block_norms(v, bid, nblk):
    return np.sqrt(np.bincount(bid, weights=np.sum(np.abs(v) ** 2, axis=(1, 2)), minlength=nblk))


def _stop_steps(hist, alpha, tol, nmr_max):
    """Sec. 3.2 exit rules applied to one block's MR residual history hist[0..nmr_max]
    (hist[0] the norm before the first step): the step count at which the block stops."""
    if hist[0] < tol:
        return 0
    for k in range(1, nmr_max + 1):
        if (k >= 4 and hist[k] > alpha * hist[k - 1]) or hist[k] > hist[k - 1] or hist[k] < tol:
            return k
    return nmr_max


def _colour_by_rules(op, r, colour, alpha, tol, nmr_max, bid, col, nblk):
    """Block solves of one colour built from the MR iteration of mr_blocks (pinned by the
    closed form of one MR step): each block's stop step comes from its own residual history
    under the exit rules, and its correction is that of mr_blocks run for exactly that many
    steps. Returns the correction, the steps per block of the colour, and the smallest
    distance of a step ratio from alpha (so that the test can refuse knife-edge cases)."""
    blocks = np.unique(bid[col == colour])
    _, _, norms = oracle.mr_blocks(op, r, BS2, colour, nmr_max, bid, col, nblk, history=True)
    hist = np.array([_block_norms(np.where((col == colour)[:, None, None], r, 0), bid, nblk)]
                    + list(norms))
    steps = np.array([_stop_steps(hist[:, b], alpha, tol, nmr_max) for b in blocks])
    margin = np.inf
    for b in blocks:
        if hist[0, b] > 0:
            margin = min(margin, np.abs(hist[1:, b] / hist[:-1, b] - alpha).min())
    chi = np.zeros_like(r)
    for s in np.unique(steps):
        if s == 0:
            continue
        part, _ = oracle.mr_blocks(op, r, BS2, colour, int(s), bid, col, nblk)
        sel = np.isin(bid, blocks[steps == s])[:, None, None]
        chi = chi + np.where(sel, part, 0)
    return chi, steps, margin


@pytest.mark.parametrize("alpha, tol_from", [(0.42, None), (0.42, 2), (0.9, 3)])
def test_adaptive_sap_steps_follow_the_exit_rules(op44, alpha, tol_from):
    """One cycle of adaptive SAP against the Sec. 3.2 rules applied to independently
    computed MR histories: exit (1) after at least 4 steps when |r_b| > alpha times its value
    one step before, (2) when |r_b| grew, (3) when |r_b| < tol; blocks below tol at the start
    take no step. The cases make blocks stop at different steps through rules (1) and (3);
    reading 'previous' as the block's initial residual, or requiring 5 steps, changes them."""
    rho = syn.gaussian_spinor(D44, 36)
    bid, col, nblk = oracle.block_ids(D44, BS2)
    rho = np.where((bid == np.unique(bid[col == 0])[1])[:, None, None], 0, rho)  # one empty block
    nmr_max = 12
    tol = 0.0
    if tol_from is not None:
        # tol between the block residuals after step tol_from: rule (3) stops some blocks early
        _, _, norms = oracle.mr_blocks(op44, rho, BS2, 0, nmr_max, bid, col, nblk, history=True)
        used = np.unique(bid[col == 0])
        h = norms[tol_from - 1][used]
        h = h[h > 0]
        tol = float(np.median(h))
    chi0, s0, m0 = _colour_by_rules(op44, rho, 0, alpha, tol, nmr_max, bid, col, nblk)
    r1 = rho - op44.dw(chi0)
    chi1, s1, m1 = _colour_by_rules(op44, r1, 1, alpha, tol, nmr_max, bid, col, nblk)
    assert min(m0, m1) > 1e-6  # no step ratio sits on the threshold
    steps_all = np.concatenate([s0, s1])
    assert (0 in s0) == (tol > 0)                    # the empty block (rule 3 at the start)
    assert len(np.unique(steps_all)) >= 3            # the rules act differently per block
    if tol_from is None:
        assert 4 in steps_all and np.any(steps_all > 4)
    else:
        assert np.any((steps_all > 0) & (steps_all < 4))  # rule (3) before rule (1) may act
    psi, cycles, steps = oracle.sap_adaptive(op44, rho, BS2, 1, nmr_max, alpha, tol)
    assert cycles == 1
    assert np.array_equal(steps[0], s0) and np.array_equal(steps[1], s1)
    want = chi0 + chi1
    assert np.abs(psi - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("m0", [-0.8, -1.5])
def test_adaptive_sap_cycles_stop_when_residual_does_not_drop(m0):
    """Sec. 3.2: the application stops after the first Schwarz cycle that did not lower |r|.
    With the MR exits switched off (alpha huge, tol 0) each cycle is a plain SAP cycle, so
    the expected cycle count is read off the residual norms of plain SAP with 1, 2, ...
    cycles (pinned by block Gauss-Seidel); for these strongly negative masses SAP stops
    converging, at cycle 3 (m0 = -0.8) or already at cycle 2 (m0 = -1.5). The cycle that
    raised |r| is kept, as the exit rules keep the MR step that triggered them."""
    op = _op(D44, m0=m0)
    rho = syn.gaussian_spinor(D44, 40)
    prev = np.linalg.norm(rho)
    expect = None
    for c in range(1, 10):
        n = np.linalg.norm(rho - op.dw(oracle.sap(op, rho, BS2, c, 4)))
        if n >= prev:
            expect = c
            break
        prev = n
    assert expect == {-0.8: 3, -1.5: 2}[m0]
    psi, cycles, steps = oracle.sap_adaptive(op, rho, BS2, 10, 4, 1e300, 0.0)
    assert cycles == expect and all(np.all(s == 4) for s in steps)
    want = oracle.sap(op, rho, BS2, expect, 4)
    assert np.abs(psi - want).max() <= 1e-12 * np.abs(want).max()


# ----------------------------------------------------------------- network

DN = (4, 2, 2, 4)


@pytest.fixture(scope="module")
def opn():
    return _op(DN, m0=-0.05, csw=1.7, seed=44)


def _rand_weights(seed, scale=0.3):
    return oracle.nn_identity_weights(seed=seed, scale=scale)


def test_nn_identity_init(opn):
    r = syn.gaussian_spinor(DN, 1)
    out, _ = oracle.nn_forward(opn, oracle.nn_identity_weights(), r)
    assert np.array_equal(out, r)


def test_nn_loss_with_identity_network(opn):
    """With the identity network (N(r) = r, pinned above) the loss is the relative squared
    distance: 0 for e = r, exactly 4 for e = -r (N(r) - e = 2 r), and |r - e|^2 / |e|^2 in
    general, with dL/d conj(out) = (r - e) / |e|^2."""
    W = oracle.nn_identity_weights()
    r = syn.gaussian_spinor(DN, 10)
    e = syn.gaussian_spinor(DN, 11)
    assert oracle.nn_loss(opn, W, r, r)[0] == 0.0
    assert abs(oracle.nn_loss(opn, W, r, -r)[0] - 4.0) < 1e-14
    L, g, _ = oracle.nn_loss(opn, W, r, e)
    ne2 = np.linalg.norm(e.reshape(-1)) ** 2
    assert abs(L - np.linalg.norm((r - e).reshape(-1)) ** 2 / ne2) < 1e-14 * L
    assert np.abs(g - (r - e) / ne2).max() < 1e-15


def test_nn_transport_adjoint_pairs(opn):
    a = syn.gaussian_spinor(DN, 2)
    b = syn.gaussian_spinor(DN, 3)
    for p in range(oracle.NPATH):
        lhs = np.vdot(b, oracle.nn_transport(opn, a, p))
        rhs = np.vdot(oracle.nn_transport_adj(opn, b, p), a)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_nn_transport_reproduces_hopping_term(opn):
    """The hop part of D is -1/2 sum_mu [(1-gamma_mu) T_{+mu} + (1+gamma_mu) T_{-mu}]."""
    psi = syn.gaussian_spinor(DN, 4)
    g = oracle.gamma()
    hop = np.zeros_like(psi)
    for mu in range(4):
        hop -= 0.5 * spin(np.eye(4) - g[mu], oracle.nn_transport(opn, psi, 1 + 2 * mu))
        hop -= 0.5 * spin(np.eye(4) + g[mu], oracle.nn_transport(opn, psi, 2 + 2 * mu))
    diag = np.einsum("xij,xj->xi", opn.A, psi.reshape(-1, 12)).reshape(psi.shape)
    assert np.abs(opn.dw(psi) - (diag + hop)).max() < 1e-13


def dirac_weights(m0, route=(3, 5)):
    """Network weights whose three layers multiply by D at c_sw = 0: layer 1 copies the input
    into channel route[0] (identity path), layer 2 maps channel route[0] to channel route[1]
    with W_0 = (4 + m0) 1, W_{+mu} = -1/2 (1 - gamma_mu), W_{-mu} = -1/2 (1 + gamma_mu), and
    layer 3 copies channel route[1] to the output."""
    g = oracle.gamma()
    a, b = route
    W1 = np.zeros((oracle.NPATH, 8, 1, 4, 4), dtype=np.complex128)
    W2 = np.zeros((oracle.NPATH, 8, 8, 4, 4), dtype=np.complex128)
    W3 = np.zeros((oracle.NPATH, 1, 8, 4, 4), dtype=np.complex128)
    W1[0, a, 0] = np.eye(4)
    W2[0, b, a] = (4.0 + m0) * np.eye(4)
    for mu in range(4):
        W2[1 + 2 * mu, b, a] = -0.5 * (np.eye(4) - g[mu])
        W2[2 + 2 * mu, b, a] = -0.5 * (np.eye(4) + g[mu])
    W3[0, 0, b] = np.eye(4)
    return [W1, W2, W3]


@pytest.mark.parametrize("bc", [-1, 1])
def test_nn_with_dirac_weights_is_the_operator(bc):
    """With the weights of dirac_weights the network is the Wilson operator without clover
    term, written independently in oracle.c: this fixes the spin index order of the weight
    matrices (gamma_1, gamma_3 are not symmetric), the direction and boundary sign of each
    transport path, and which index of W is the output channel (the copy goes through
    channels 3 and 5, so swapped channel indices give zero)."""
    dims = (4, 2, 4, 6)
    su3, th = syn.gauge_field(dims, 0.3, 0.1, 46)
    op = oracle.Operator(dims, su3, th, -0.05, 0.0, bc)
    r = syn.gaussian_spinor(dims, 10)
    out, _ = oracle.nn_forward(op, dirac_weights(-0.05), r)
    want = op.dw(r)
    assert np.abs(out - want).max() <= 1e-13 * np.abs(want).max()
    # gamma_5 D gamma_5 = D^+ with the projector signs swapped
    Wd = dirac_weights(-0.05)
    for p in range(1, oracle.NPATH):
        Wd[1][p, 5, 3] = -np.eye(4) - Wd[1][p, 5, 3]  # -1/2 (1 -+ g) -> -1/2 (1 +- g)
    out, _ = oracle.nn_forward(op, Wd, r)
    want = op.dw_dag(r)
    assert np.abs(out - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("dims, bc", [((4, 2, 4, 6), -1), ((6, 4, 4, 4), 1)])
def test_nn_at_sites_equals_full_forward(dims, bc):
    """The per-site network evaluation (its own transport code, limited to the receptive
    field) agrees with the full forward pass at every site and on a scrambled subset."""
    su3, th = syn.gauge_field(dims, 0.3, 0.1, 47)
    op = oracle.Operator(dims, su3, th, -0.05, 1.7, bc)
    W = _rand_weights(3)
    r = syn.gaussian_spinor(dims, 11)
    want, _ = oracle.nn_forward(op, W, r)
    got = oracle.nn_at_sites(dims, bc, op.u, W, r, np.arange(op.V))
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    sub = np.random.default_rng(2).permutation(op.V)[:29]
    got = oracle.nn_at_sites(dims, bc, op.u, W, r, sub)
    assert np.abs(got - want[sub]).max() <= 1e-13 * np.abs(want).max()


def test_nn_linear_and_equivariant():
    dims = (4, 2, 2, 4)
    su3, th = syn.gauge_field(dims, 0.3, 0.1, 45)
    op = oracle.Operator(dims, su3, th, -0.05, 1.7, -1)
    W = _rand_weights(1)
    a, b = syn.gaussian_spinor(dims, 5), syn.gaussian_spinor(dims, 6)
    na, _ = oracle.nn_forward(op, W, a)
    nb_, _ = oracle.nn_forward(op, W, b)
    nab, _ = oracle.nn_forward(op, W, a + 2j * b)
    assert np.abs(nab - (na + 2j * nb_)).max() < 1e-12 * np.abs(nab).max()
    G = syn.random_gauge_transform(dims, 7)
    nbm = oracle.neighbours(dims)
    ug = np.einsum("xij,xmjk,xmlk->xmil", G, op.u, np.conj(G[nbm[:, 0::2]]))
    thg = np.angle(np.linalg.det(ug)) / 3.0
    opg = oracle.Operator(dims, ug * np.exp(-1j * thg)[..., None, None], thg, -0.05, 1.7, -1)
    Ga = np.einsum("xij,xsj->xsi", G, a)
    lhs, _ = oracle.nn_forward(opg, W, Ga)
    rhs = np.einsum("xij,xsj->xsi", G, na)
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


def test_nn_gradients_finite_differences(opn):
    W = _rand_weights(2, 0.2)
    r = syn.gaussian_spinor(DN, 8)
    e = syn.gaussian_spinor(DN, 9)
    L, g, acts = oracle.nn_loss(opn, W, r, e)
    grads, gin = oracle.nn_backward(opn, W, acts, g)
    rng = np.random.default_rng(0)
    h = 1e-6
    for l in range(3):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in W[l].shape)
            for unit, part in ((1.0, "re"), (1j, "im")):
                Wp = [w.copy() for w in W]
                Wm = [w.copy() for w in W]
                Wp[l][idx] += unit * h
                Wm[l][idx] -= unit * h
                fd = (oracle.nn_loss(opn, Wp, r, e)[0] - oracle.nn_loss(opn, Wm, r, e)[0]) / (2 * h)
                an = grads[l][idx].real if part == "re" else grads[l][idx].imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (l, idx, part, fd, an)
    # input gradient: dL/dRe r + i dL/dIm r = 2 gin
    for _ in range(4):
        j = tuple(rng.integers(0, s) for s in r.shape)
        rp, rm = r.copy(), r.copy()
        rp[j] += h
        rm[j] -= h
        fd = (oracle.nn_loss(opn, W, rp, e)[0] - oracle.nn_loss(opn, W, rm, e)[0]) / (2 * h)
        assert abs(fd - 2 * gin[j].real) <= 1e-6 * max(1.0, abs(fd))


# ---------------------------------------------------------------- even-odd reduction

def _eo_index(dims):
    par = np.repeat(oracle.site_parity(dims), 12)
    return np.flatnonzero(par == 0), np.flatnonzero(par == 1)


def test_schur_equals_dense_schur_complement(op44, dense44):
    """Column by column, the oracle's D^ equals D_EE - D_EO D_OO^-1 D_OE formed from the
    brute-force dense matrix."""
    E, O = _eo_index(D44)
    S = dense44[np.ix_(E, E)] - dense44[np.ix_(E, O)] @ np.linalg.solve(
        dense44[np.ix_(O, O)], dense44[np.ix_(O, E)])
    sc = oracle.Schur(op44)
    e = np.zeros(op44.V * 12, dtype=np.complex128)
    rng = np.random.default_rng(5)
    for j in rng.choice(len(E), 48, replace=False):
        e[E[j]] = 1.0
        col = sc.apply(e).reshape(-1)
        e[E[j]] = 0.0
        assert np.abs(col[E] - S[:, j]).max() < 1e-13
        assert np.abs(col[O]).max() == 0.0
    # a random even field at once
    v = rng.standard_normal(len(E)) + 1j * rng.standard_normal(len(E))
    f = np.zeros(op44.V * 12, dtype=np.complex128)
    f[E] = v
    assert np.abs(sc.apply(f).reshape(-1)[E] - S @ v).max() < 1e-12


def test_schur_determinant_identity():
    """det D = det D_OO det D^ (block LU); a swapped or mis-signed coupling breaks it."""
    dims = (4, 2, 2, 2)
    op = _op(dims, m0=-0.1, csw=1.7, eps=0.4, seed=21)
    M = oracle.dense_matrix(op)
    E, O = _eo_index(dims)
    sc = oracle.Schur(op)
    n = len(E)
    S = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(op.V * 12, dtype=np.complex128)
    for j in range(n):
        e[E[j]] = 1.0
        S[:, j] = sc.apply(e).reshape(-1)[E]
        e[E[j]] = 0.0
    s_full, l_full = np.linalg.slogdet(M)
    s_oo, l_oo = np.linalg.slogdet(M[np.ix_(O, O)])
    s_s, l_s = np.linalg.slogdet(S)
    assert abs(l_full - (l_oo + l_s)) < 1e-10
    assert abs(s_full - s_oo * s_s) < 1e-10


def test_schur_reconstructs_the_full_solution(op44, dense44):
    """For x = D^-1 eta: D^ x_e = eta^_e, and the odd rows give back x_o."""
    eta = syn.gaussian_spinor(D44, 77)
    x = np.linalg.solve(dense44, eta.reshape(-1)).reshape(eta.shape)
    sc = oracle.Schur(op44)
    lhs = sc.apply(x)
    rhs = sc.source(eta)
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()
    back = sc.solve_full(eta, x)
    assert np.abs(back - x).max() < 1e-12 * np.abs(x).max()


def test_schur_gamma5_hermitian(op44):
    sc = oracle.Schur(op44)
    g5 = np.diag([1.0, 1.0, -1.0, -1.0])
    v = syn.gaussian_spinor(D44, 78)
    lhs = spin(g5, sc.apply(spin(g5, v)))
    assert np.abs(lhs - sc.apply_dag(v)).max() < 1e-13
    w = syn.gaussian_spinor(D44, 79)
    ev = np.where(sc.even, w, 0)
    assert abs(np.vdot(ev, sc.apply(v)) - np.vdot(sc.apply_dag(ev), v)) < 1e-11


def test_cgne_schur_solves_the_reduced_normal_equations(op44, dense44):
    E, _ = _eo_index(D44)
    sc = oracle.Schur(op44)
    eta = syn.gaussian_spinor(D44, 80)
    x, st = oracle.cgne_schur(sc, eta, 1e-10, 2000)
    assert st > 0
    r = np.where(sc.even, eta, 0) - sc.normal(x)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(np.where(sc.even, eta, 0))
    # against the dense normal equations of the dense Schur complement
    O = np.setdiff1d(np.arange(op44.V * 12), E)
    S = dense44[np.ix_(E, E)] - dense44[np.ix_(E, O)] @ np.linalg.solve(
        dense44[np.ix_(O, O)], dense44[np.ix_(O, E)])
    xd = np.linalg.solve(S.conj().T @ S, eta.reshape(-1)[E])
    assert np.linalg.norm(x.reshape(-1)[E] - xd) <= 1e-7 * np.linalg.norm(xd)
    # the reduced system needs fewer CG steps than the full normal equations
    _, st_full = oracle.cgne(op44, eta, 1e-10, 2000)
    assert st < st_full, (st, st_full)


# ---------------------------------------------------------------- SAP with even-odd blocks

def test_sap_eo_cycle_is_block_gauss_seidel(op44, dense44):
    """Exact block solves do not depend on how they are reached: with MR on the reduced
    block operator run to convergence, one cycle is the same block Gauss-Seidel sweep
    (dense block inverses) as for the plain block solver."""
    rho = syn.gaussian_spinor(D44, 37)
    bid, col, _ = oracle.block_ids(D44, BS2)
    c12 = np.repeat(col, 12)
    b, w = c12 == 0, c12 == 1
    r = rho.reshape(-1)
    psi = np.zeros_like(r)
    psi[b] = np.linalg.solve(dense44[np.ix_(b, b)], r[b])
    res = r - dense44 @ psi
    psi[w] = np.linalg.solve(dense44[np.ix_(w, w)], res[w])
    got = oracle.sap_eo(op44, rho, BS2, 1, 80).reshape(-1)
    assert np.linalg.norm(got - psi) <= 1e-9 * np.linalg.norm(psi)


def test_sap_eo_block_residual_is_even(op44):
    """After a colour's reduced block solves the odd components of the block residual
    vanish (chi_o solves the odd rows exactly)."""
    rho = syn.gaussian_spinor(D44, 38)
    bid, col, _ = oracle.block_ids(D44, BS2)
    psi = oracle.sap_eo(op44, rho, BS2, 1, 3)
    # only the colour-1 blocks were solved last; recompute their block residual
    par = oracle.site_parity(D44)
    mask1 = (col == 1)
    # residual of the colour-1 blocks after the sweep: rho - D psi restricted to them,
    # minus the part that the colour-0 update changed afterwards (none: colour 1 is last)
    r = rho - op44.dw(psi)
    assert np.abs(r[mask1 & (par == 1)]).max() < 1e-12 * np.abs(rho).max()


def test_sap_eo_fewer_steps_than_plain_blocks(op44):
    """The reduced block problems converge faster: for the same nmr the preconditioned
    residual |rho - D M rho| is smaller than with plain block MR."""
    rho = syn.gaussian_spinor(D44, 39)
    a = np.linalg.norm(rho - op44.dw(oracle.sap_eo(op44, rho, BS2, 2, 3)))
    b = np.linalg.norm(rho - op44.dw(oracle.sap(op44, rho, BS2, 2, 3)))
    assert a < b, (a, b)


# ---------------------------------------------------------------- rounding bound of D^

def _round_to(x, mant):
    """Round to `mant` fraction bits, to nearest (the 16-bit formats' significands)."""
    if np.iscomplexobj(x):
        return _round_to(x.real, mant) + 1j * _round_to(x.imag, mant)
    m, e = np.frexp(x)
    return np.ldexp(np.round(m * 2.0 ** (mant + 1)) / 2.0 ** (mant + 1), e)


@pytest.mark.parametrize("mant", [10, 7])
def test_schur_rounding_bound_holds_for_emulated_storage(mant):
    """The first-order bound the GPU test of the reduced operator uses (schur_bound.py)
    covers the errors of the same computation with every stored number rounded to a
    16-bit significand (10 fraction bits: binary16, 7: bfloat16), emulated here in FP64."""
    import sys, os
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from schur_bound import schur_error_bound
    dims = (6, 4, 6, 10)
    su3, th = syn.gauge_field(dims, 0.3, 0.1, 61)
    op = oracle.Operator(dims, su3, th, -0.05, 1.7, -1)
    sc = oracle.Schur(op)
    v = syn.gaussian_spinor(dims, 62)
    u = 2.0 ** -(mant + 1)
    for dag in (False, True):
        bound, out = schur_error_bound(op, sc, v, u, dag=dag)
        em = oracle.Operator(dims, su3, th, -0.05, 1.7, -1)
        r0, r1 = _round_to(op.u[..., 0, :], mant), _round_to(op.u[..., 1, :], mant)
        d = _round_to(np.linalg.det(op.u), mant)
        em.u = np.ascontiguousarray(np.stack([r0, r1, d[..., None] * np.conj(np.cross(r0, r1))],
                                             axis=-2))
        em.A = np.ascontiguousarray(_round_to(op.A, mant))
        esc = oracle.Schur(em)
        esc.Ainv = _round_to(sc.Ainv, mant)
        pe = _round_to(np.where(sc.even, v, 0), mant)
        fwd = em.dw_dag if dag else em.dw
        y = fwd(pe)
        t = _round_to(np.where(sc.odd, esc._ainv(np.where(sc.odd, y, 0)), 0), mant)
        got = _round_to(np.where(sc.even, y - fwd(t), 0), mant)
        err = np.abs(got - out)[sc.even[:, 0, 0]]
        b = bound[sc.even[:, 0, 0]]
        assert np.all(err <= b), float((err / np.maximum(b, 1e-300)).max())
        assert (err / np.maximum(b, 1e-300)).max() > 0.02  # and it is not vacuous
