"""FP64 CPU oracle for the Wilson-clover operator and its solvers.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py``, never by the product library. It shares no code with
the HIP path; the two meet only in the seeded inputs of ``paper_2202_07388_amd.synthetic``.

Contents, each written from its definition (stencil loops live in ``oracle.c``):

* ``Operator``: D and D^+ (explicit adjoint stencil), block-restricted D_b, clover term;
* ``dense_matrix``: brute-force D as a dense matrix, for tiny lattices;
* ``cgne``: textbook conjugate gradient on D^+ D (Sec. 2 of the paper: ``cgne()``),
  returning the number of CG steps (``status``) and the diagnostics of the paper's
  Fig. 1 (exact residual, recursive residual, A-orthogonality of successive directions);
* ``fgcr``: flexible GCR with restarts (Sec. 3.1, Table 2 settings res, nmx, nkv);
* ``sap`` / ``mr_blocks``: Schwarz alternating procedure (Sec. 3, Fig. 2 and 3): chessboard
  blocks, grey then white, ``nmr`` minimal-residual steps per block, ``ncy`` cycles;
* ``sap_adaptive``: the adaptive variant of Sec. 3.2; ``sap_eo``: SAP with even-odd
  reduced block solves;
* ``Schur`` / ``cgne_schur``: the even-odd reduced operator A_ee - D_eo A_oo^-1 D_oe and
  CG on its normal equations;
* ``nn_*``: a gauge-covariant linear network of parallel-transport layers, forward and
  analytic adjoint (not from the paper).

Parity status: see each function's docstring; every function here is pinned by the CPU
tests. The U(1) charge in the clover term (q = 1, a single c_sw for the combined U(3)
link) is a reading of the paper, which fixes neither; its arithmetic is pinned by the
constant abelian flux. Mixed-precision and learned solves have no counterpart here (their
solutions are judged by the FP64 true residual of this operator).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


_NATIVE = os.path.join(_HERE, "liboracle_native.so")


def build(force: bool = False, native: bool = False) -> str:
    """Compile oracle.c with gcc (C99, -O3, OpenMP over sites): liboracle.so for any
    x86-64 host, or with native=True liboracle_native.so tuned for the host that builds
    it (-march=native; built and used on the machine that times the oracle)."""
    out = _NATIVE if native else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        flags = ["-O3", "-std=gnu99", "-fopenmp", "-fPIC", "-shared"]
        if native:
            flags.append("-march=native")
        subprocess.check_call(["gcc", *flags, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


def use_native_build():
    """Switch this process's oracle to the -march=native build (before first use)."""
    global _lib, _LIB
    if _lib is not None and _LIB == _NATIVE:
        return
    if _lib is not None:
        raise RuntimeError("oracle already loaded; switch before the first call")
    build(force=True, native=True)  # always for the host at hand
    _LIB = _NATIVE


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's site loops."""
    lib().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def lib():
    global _lib
    if _lib is None:
        if _LIB != _NATIVE:
            build()
        L = ctypes.CDLL(_LIB)
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_max_threads.restype = ctypes.c_int
        P = ctypes.c_void_p
        L.oracle_gamma.argtypes = [P]
        L.oracle_neighbours.argtypes = [P, P]
        L.oracle_clover.argtypes = [P, P, ctypes.c_double, ctypes.c_double, P]
        for f in (L.oracle_dw, L.oracle_dw_dag):
            f.argtypes = [P, ctypes.c_int, P, P, P, P]
        L.oracle_dw_blocks.argtypes = [P, P, ctypes.c_int, P, P, P, P]
        L.oracle_u3_links.argtypes = [ctypes.c_long, P, P, P]
        L.oracle_dw_at.argtypes = [P, ctypes.c_int, P, ctypes.c_double, ctypes.c_double, P, P,
                                   ctypes.c_long, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(d):
    return np.ascontiguousarray(np.asarray(d, dtype=np.int32))


def gamma() -> np.ndarray:
    out = np.zeros((4, 4, 4), dtype=np.complex128)
    lib().oracle_gamma(_p(out))
    return out


def neighbours(dims) -> np.ndarray:
    V = int(np.prod(dims))
    nb = np.zeros((V, 8), dtype=np.int64)
    lib().oracle_neighbours(_p(_dims(dims)), _p(nb))
    return nb


def u3_links(su3: np.ndarray, theta: np.ndarray) -> np.ndarray:
    su3 = np.ascontiguousarray(su3, dtype=np.complex128)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    u = np.empty_like(su3)
    lib().oracle_u3_links(su3.shape[0], _p(su3), _p(theta), _p(u))
    return u


def clover(dims, u: np.ndarray, m0: float, csw: float) -> np.ndarray:
    """A(x) as [V, 12, 12] (index spin*3 + colour)."""
    V = int(np.prod(dims))
    A = np.zeros((V, 12, 12), dtype=np.complex128)
    lib().oracle_clover(_p(_dims(dims)), _p(np.ascontiguousarray(u)), m0, csw, _p(A))
    return A


class Operator:
    """The Wilson-clover operator on one gauge field (links kept as full U(3) matrices)."""

    def __init__(self, dims, su3, theta, m0, csw, bc_t=-1):
        self.dims = tuple(int(v) for v in dims)
        self.V = int(np.prod(self.dims))
        self.bc_t = int(bc_t)
        self.m0, self.csw = float(m0), float(csw)
        self.u = u3_links(su3, theta)
        self.A = clover(self.dims, self.u, self.m0, self.csw)
        self._d = _dims(self.dims)

    def _apply(self, fn, psi, *extra):
        psi = np.ascontiguousarray(psi, dtype=np.complex128).reshape(self.V, 4, 3)
        out = np.empty_like(psi)
        fn(_p(self._d), *extra, self.bc_t, _p(self.u), _p(self.A), _p(psi), _p(out))
        return out

    def dw(self, psi):
        return self._apply(lib().oracle_dw, psi)

    def dw_dag(self, psi):
        return self._apply(lib().oracle_dw_dag, psi)

    def dw_blocks(self, psi, bs):
        return self._apply(lib().oracle_dw_blocks, psi, _p(_dims(bs)))

    def normal(self, psi):
        return self.dw_dag(self.dw(psi))


def dw_at_sites(dims, bc_t, u, m0, csw, psi, sites):
    """(D psi)(x) for the listed lexicographic sites only ([n, 4, 3]); the clover term is
    built at those sites from its definition. For sampling lattices too large for a full
    oracle sweep."""
    sites = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.zeros((len(sites), 4, 3), dtype=np.complex128)
    lib().oracle_dw_at(_p(_dims(dims)), int(bc_t), _p(np.ascontiguousarray(u)), float(m0),
                       float(csw), _p(psi), _p(sites), len(sites), _p(out))
    return out


def dense_matrix(op: Operator, which: str = "dw") -> np.ndarray:
    """Brute force: column j of D is D applied to the j-th unit vector."""
    n = op.V * 12
    f = {"dw": op.dw, "dag": op.dw_dag}[which]
    M = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = f(e).reshape(-1)
        e[j] = 0.0
    return M


def dense_block_matrix(op: Operator, bs) -> np.ndarray:
    n = op.V * 12
    M = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = op.dw_blocks(e, bs).reshape(-1)
        e[j] = 0.0
    return M


def _dot(a, b) -> complex:
    return complex(np.vdot(a.reshape(-1), b.reshape(-1)))


def _norm(a) -> float:
    return float(np.sqrt(np.vdot(a.reshape(-1), a.reshape(-1)).real))


# --------------------------------------------------------------------------- CGNE

def cgne(op: Operator, eta, res: float, nmx: int, history: bool = False):
    """Conjugate gradient on A = D^+ D from psi = 0 (paper Sec. 2, ``cgne()``).

    Stops when the recursive residual |r| <= res*|eta|, then confirms with the true
    residual eta - D^+ D psi and continues from it if the check fails. ``status`` is the
    number of CG steps, -1 when nmx steps did not suffice. The recursive residual uses
    r_i = r_{i-1} - alpha_{i-1} A p_{i-1} (the sign of Fig. 1's caption is a convention).
    Diagnostics per step (Fig. 1): exact relative residual, recursive relative residual,
    and p_{i-1}^+ A p_i.
    """
    eta = np.asarray(eta, dtype=np.complex128).reshape(op.V, 4, 3)
    neta = _norm(eta)
    x = np.zeros_like(eta)
    r = eta.copy()
    p = r.copy()
    rr = _norm(r) ** 2
    hist = {"exact": [], "recursive": [], "a_orth": []}
    q_prev = None
    status = 0
    while True:
        q = op.dw(p)
        w = op.dw_dag(q)
        pap = _norm(q) ** 2
        if history and q_prev is not None:
            hist["a_orth"].append(_dot(q_prev, q))
        q_prev = q
        alpha = rr / pap
        x = x + alpha * p
        r = r - alpha * w
        rr_new = _norm(r) ** 2
        status += 1
        if history:
            hist["exact"].append(_norm(eta - op.normal(x)) / neta)
            hist["recursive"].append(np.sqrt(rr_new) / neta)
        if np.sqrt(rr_new) <= res * neta:
            rt = eta - op.normal(x)
            if _norm(rt) <= res * neta:
                break
            r = rt
            rr_new = _norm(r) ** 2
        if status >= nmx:
            status = -1
            break
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
    return (x, status, hist) if history else (x, status)


# --------------------------------------------------------------------------- even-odd

def site_parity(dims) -> np.ndarray:
    """(x0 + x1 + x2 + x3) mod 2 per lexicographic site."""
    return np.indices(tuple(dims)).reshape(4, -1).sum(axis=0) % 2


class Schur:
    """The even-odd reduced operator D^ = A_ee - D_eo A_oo^-1 D_oe on even-site fields
    (the matrix of the paper's Sec. 3 is even-odd ordered, Fig. 3 left; its even-even
    Schur complement), written from the blocks of D itself:

    * (D (psi_e, 0))_even = A_ee psi_e and (D (psi_e, 0))_odd = D_oe psi_e, since no hop
      joins two sites of one parity;
    * (D (0, t))_even = D_eo t;
    * A_oo^-1 is the inverse of each odd site's 12 x 12 clover matrix.

    Fields are full-size [V, 4, 3] arrays; odd components of the input are ignored and
    those of the output are zero. D^+ is built the same way from D^+ (A is Hermitian).
    """

    def __init__(self, op: Operator):
        self.op = op
        par = site_parity(op.dims)
        self.even = (par == 0)[:, None, None]
        self.odd = (par == 1)[:, None, None]
        self.Ainv = np.linalg.inv(op.A)

    def _ainv(self, y):
        return np.einsum("sab,sb->sa", self.Ainv, y.reshape(-1, 12)).reshape(y.shape)

    def _apply(self, fwd, psi):
        psi = np.asarray(psi, dtype=np.complex128).reshape(self.op.V, 4, 3)
        y = fwd(np.where(self.even, psi, 0))
        t = np.where(self.odd, self._ainv(np.where(self.odd, y, 0)), 0)
        z = fwd(t)
        return np.where(self.even, y - z, 0)

    def apply(self, psi):
        return self._apply(self.op.dw, psi)

    def apply_dag(self, psi):
        return self._apply(self.op.dw_dag, psi)

    def normal(self, psi):
        return self.apply_dag(self.apply(psi))

    def solve_full(self, eta, x_even):
        """Given the even part x_e of the solution of D x = eta, the odd part follows
        from the odd rows: x_o = A_oo^-1 (eta_o - D_oe x_e)."""
        eta = np.asarray(eta, dtype=np.complex128).reshape(self.op.V, 4, 3)
        xe = np.where(self.even, np.asarray(x_even).reshape(self.op.V, 4, 3), 0)
        y = self.op.dw(xe)
        xo = np.where(self.odd, self._ainv(np.where(self.odd, eta - y, 0)), 0)
        return xe + xo

    def source(self, eta):
        """eta^_e = eta_e - D_eo A_oo^-1 eta_o: D^ x_e = eta^_e for the even part of the
        solution of D x = eta."""
        eta = np.asarray(eta, dtype=np.complex128).reshape(self.op.V, 4, 3)
        t = np.where(self.odd, self._ainv(np.where(self.odd, eta, 0)), 0)
        return np.where(self.even, eta - self.op.dw(t), 0)


def cgne_schur(sc: Schur, eta, res: float, nmx: int):
    """Textbook CG on D^+ D^ over even-site fields from x = 0, stopping when the true
    residual |eta_e - D^+ D^ x| <= res |eta_e| (checked when the recursive one is)."""
    eta = np.where(sc.even, np.asarray(eta, dtype=np.complex128).reshape(sc.op.V, 4, 3), 0)
    neta = _norm(eta)
    x = np.zeros_like(eta)
    r = eta.copy()
    p = r.copy()
    rr = _norm(r) ** 2
    status = 0
    while True:
        q = sc.apply(p)
        alpha = rr / _norm(q) ** 2
        x = x + alpha * p
        r = r - alpha * sc.apply_dag(q)
        rr_new = _norm(r) ** 2
        status += 1
        if np.sqrt(rr_new) <= res * neta:
            rt = eta - sc.normal(x)
            if _norm(rt) <= res * neta:
                break
            r = rt
            rr_new = _norm(r) ** 2
        if status >= nmx:
            status = -1
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, status


# --------------------------------------------------------------------------- FGCR

def fgcr(op: Operator, eta, res: float, nmx: int, nkv: int, precond=None,
         history: bool = False):
    """Flexible GCR with restart after nkv Krylov vectors (paper Sec. 3.1, Table 2).

    psi = 0, rho = eta. Within a cycle, for k < nkv: phi_k = M(rho); chi_k = D phi_k;
    Gram-Schmidt of chi_k against chi_0..chi_{k-1} (a_lk = chi_l^+ chi_k, chi_k -= a_lk
    chi_l), b_k = |chi_k|, chi_k /= b_k, c_k = chi_k^+ rho, rho -= c_k chi_k. At the end of
    a cycle (nkv vectors, convergence or nmx), solve the upper-triangular R alpha = c
    (R_lk = a_lk, R_kk = b_k), psi += sum alpha_l phi_l and recompute rho = eta - D psi
    in FP64 (the restart step). ``precond`` is M (None: identity). Returns psi, status
    (GCR steps, -1 when nmx steps did not suffice) and, if asked, the recursive residual
    norm after every step.
    """
    eta = np.asarray(eta, dtype=np.complex128).reshape(op.V, 4, 3)
    M = precond if precond is not None else (lambda v: v.copy())
    neta = _norm(eta)
    tol = res * neta
    psi = np.zeros_like(eta)
    rho = eta.copy()
    status = 0
    hist = []
    while True:
        phis, chis = [], []
        R = np.zeros((nkv, nkv), dtype=np.complex128)
        c = np.zeros(nkv, dtype=np.complex128)
        k = 0
        rn = _norm(rho)
        while k < nkv and status < nmx and rn > tol:
            phi = M(rho)
            chi = op.dw(phi)
            for l in range(k):
                a = _dot(chis[l], chi)
                R[l, k] = a
                chi = chi - a * chis[l]
            b = _norm(chi)
            R[k, k] = b
            chi = chi / b
            c[k] = _dot(chi, rho)
            rho = rho - c[k] * chi
            phis.append(phi)
            chis.append(chi)
            k += 1
            status += 1
            rn = _norm(rho)
            hist.append(rn / neta)
        if k > 0:
            alpha = _back_substitute(R[:k, :k], c[:k])
            for l in range(k):
                psi = psi + alpha[l] * phis[l]
            rho = eta - op.dw(psi)
            rn = _norm(rho)
        if rn <= tol:
            break
        if status >= nmx:
            status = -1
            break
    return (psi, status, hist) if history else (psi, status)


def _back_substitute(R, c):
    n = len(c)
    a = np.zeros(n, dtype=np.complex128)
    for i in range(n - 1, -1, -1):
        s = c[i] - sum(R[i, j] * a[j] for j in range(i + 1, n))
        a[i] = s / R[i, i]
    return a


# --------------------------------------------------------------------------- SAP

def block_ids(dims, bs):
    """Linear block index and block colour (sum of block coordinates mod 2) per site."""
    x = np.indices(tuple(dims)).reshape(4, -1)
    nb = [dims[m] // bs[m] for m in range(4)]
    b = [x[m] // bs[m] for m in range(4)]
    bid = ((b[0] * nb[1] + b[1]) * nb[2] + b[2]) * nb[3] + b[3]
    colour = (b[0] + b[1] + b[2] + b[3]) % 2
    return bid, colour, int(np.prod(nb))


def _block_sum(vals_per_site, bid, nblk):
    re = np.bincount(bid, weights=vals_per_site.real, minlength=nblk)
    im = np.bincount(bid, weights=vals_per_site.imag, minlength=nblk)
    return re + 1j * im


def mr_blocks(op: Operator, r, bs, colour: int, nmr: int, bid=None, col=None,
              nblk=None, history=False):
    """nmr minimal-residual steps from zero on every block of one colour at once.

    For each block b: v = D_b r_b, omega = (v^+ r_b)/(v^+ v), chi_b += omega r_b,
    r_b -= omega v (paper Sec. 3: the block problems D_i chi = r_i are solved
    approximately by MR). Returns chi (zero outside the colour) and the final block
    residuals r_b.
    """
    if bid is None:
        bid, col, nblk = block_ids(op.dims, bs)
    mask = (col == colour)[:, None, None]
    rb = np.where(mask, r, 0)
    chi = np.zeros_like(rb)
    norms = []
    for _ in range(nmr):
        v = np.where(mask, op.dw_blocks(rb, bs), 0)
        num = _block_sum(np.sum(np.conj(v) * rb, axis=(1, 2)), bid, nblk)
        den = _block_sum(np.sum(np.abs(v) ** 2, axis=(1, 2)).astype(np.complex128), bid,
                         nblk).real
        omega = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
        w = omega[bid][:, None, None]
        chi = chi + w * rb
        rb = rb - w * v
        if history:
            norms.append(np.sqrt(_block_sum(np.sum(np.abs(rb) ** 2, axis=(1, 2))
                                            .astype(np.complex128), bid, nblk).real))
    return (chi, rb, norms) if history else (chi, rb)


def sap(op: Operator, rho, bs, ncy: int, nmr: int):
    """Schwarz alternating procedure (paper Sec. 3, Fig. 2 and 3) as a preconditioner.

    psi = 0, r = rho. One cycle solves all colour-0 ("grey"/"black") blocks, then all
    colour-1 ("white") blocks, each approximately by nmr MR steps on the block-restricted
    operator D_b (Dirichlet: hops leaving the block dropped), adds the block solutions to
    psi and recomputes the full residual r = rho - D psi after each colour. ncy = 0
    returns rho unchanged (no preconditioning, the (0, 0) setting).
    """
    rho = np.asarray(rho, dtype=np.complex128).reshape(op.V, 4, 3)
    if ncy == 0:
        return rho.copy()
    bid, col, nblk = block_ids(op.dims, bs)
    psi = np.zeros_like(rho)
    r = rho.copy()
    for _ in range(ncy):
        for colour in (0, 1):
            chi, _rb = mr_blocks(op, r, bs, colour, nmr, bid, col, nblk)
            psi = psi + chi
            r = rho - op.dw(psi)
    return psi


def sap_eo(op: Operator, rho, bs, ncy: int, nmr: int):
    """SAP whose block problems are solved through their even-odd reduction (the block
    matrix is even-odd ordered like the whole lattice, Sec. 3 / Fig. 3 left): for the
    block residual r = (r_e, r_o) and the Dirichlet block operator D_b,

        r^_e = r_e - D_eo^b A_oo^-1 r_o,
        chi_e = nmr MR steps from 0 on D^_b = A_ee - D_eo^b A_oo^-1 D_oe^b with source r^_e,
        chi_o = A_oo^-1 (r_o - D_oe^b chi_e),

    then psi += chi and the full residual is recomputed after each colour, as in ``sap``.
    The blocks of D_b come from the block-restricted operator itself:
    D_b (x_e, 0) = (A_ee x_e, D_oe^b x_e) and D_b (0, t) = (D_eo^b t, A_oo t).
    """
    rho = np.asarray(rho, dtype=np.complex128).reshape(op.V, 4, 3)
    if ncy == 0:
        return rho.copy()
    bid, col, nblk = block_ids(op.dims, bs)
    par = site_parity(op.dims)
    even = (par == 0)[:, None, None]
    odd = (par == 1)[:, None, None]
    ainv = np.linalg.inv(op.A)

    def inv_odd(y):
        return np.where(odd, np.einsum("sab,sb->sa", ainv, y.reshape(-1, 12)).reshape(y.shape), 0)

    def schur_b(x):  # D^_b on even fields (zero elsewhere)
        y = op.dw_blocks(np.where(even, x, 0), bs)
        z = op.dw_blocks(inv_odd(y), bs)
        return np.where(even, y - z, 0)

    psi = np.zeros_like(rho)
    r = rho.copy()
    for _ in range(ncy):
        for colour in (0, 1):
            mask = (col == colour)[:, None, None]
            rb = np.where(mask, r, 0)
            rhat = np.where(even, rb - op.dw_blocks(inv_odd(rb), bs), 0)
            chi_e = np.zeros_like(rb)
            res = rhat
            for _k in range(nmr):
                v = np.where(mask, schur_b(res), 0)
                num = _block_sum(np.sum(np.conj(v) * res, axis=(1, 2)), bid, nblk)
                den = _block_sum(np.sum(np.abs(v) ** 2, axis=(1, 2)).astype(np.complex128), bid,
                                 nblk).real
                omega = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
                w = omega[bid][:, None, None]
                chi_e = chi_e + w * res
                res = res - w * v
            chi_o = inv_odd(np.where(odd, rb - op.dw_blocks(chi_e, bs), 0))
            psi = psi + np.where(mask, chi_e + chi_o, 0)
            r = rho - op.dw(psi)
    return psi


def sap_adaptive(op: Operator, rho, bs, ncy_max: int, nmr_max: int, alpha: float,
                 tol: float):
    """Adaptive SAP (paper Sec. 3.2).

    Cycles stop when a cycle did not lower |r| (at least one cycle runs) or after ncy_max.
    Each block's MR loop stops (1) after at least 4 steps when |r_b| > alpha * (|r_b| of
    the previous step), (2) at once when |r_b| grew over the previous step, (3) when
    |r_b| < tol (tol = res |eta| / n_b), or after nmr_max steps. The step that triggered
    an exit is kept. Returns psi and the list of (cycles, per-block MR step counts).
    """
    rho = np.asarray(rho, dtype=np.complex128).reshape(op.V, 4, 3)
    bid, col, nblk = block_ids(op.dims, bs)
    psi = np.zeros_like(rho)
    r = rho.copy()
    rn = _norm(r)
    steps = []
    cycles = 0
    for _ in range(ncy_max):
        for colour in (0, 1):
            mask = (col == colour)[:, None, None]
            rb = np.where(mask, r, 0)
            chi = np.zeros_like(rb)
            prev = np.sqrt(_block_sum(np.sum(np.abs(rb) ** 2, axis=(1, 2))
                                      .astype(np.complex128), bid, nblk).real)
            active = np.zeros(nblk, dtype=bool)
            active[np.unique(bid[col == colour])] = True
            active &= prev >= tol
            nsteps = np.zeros(nblk, dtype=np.int64)
            for k in range(nmr_max):
                if not active.any():
                    break
                act = active[bid][:, None, None] & mask
                v = np.where(act, op.dw_blocks(np.where(act, rb, 0), bs), 0)
                num = _block_sum(np.sum(np.conj(v) * rb, axis=(1, 2)), bid, nblk)
                den = _block_sum(np.sum(np.abs(v) ** 2, axis=(1, 2)).astype(np.complex128),
                                 bid, nblk).real
                omega = np.where(active & (den > 0), num / np.where(den > 0, den, 1.0), 0.0)
                w = omega[bid][:, None, None]
                chi = chi + w * rb
                rb = rb - w * v
                nsteps += active
                cur = np.sqrt(_block_sum(np.sum(np.abs(rb) ** 2, axis=(1, 2))
                                         .astype(np.complex128), bid, nblk).real)
                stop = ((k + 1 >= 4) & (cur > alpha * prev)) | (cur > prev) | (cur < tol)
                active &= ~stop
                prev = np.where(active, cur, prev)
            steps.append(nsteps[np.unique(bid[col == colour])])
            psi = psi + chi
            r = rho - op.dw(psi)
        cycles += 1
        rn_new = _norm(r)
        if rn_new >= rn:
            break
        rn = rn_new
    return psi, cycles, steps


# --------------------------------------------------------------------------- NN

NPATH = 9  # identity, then +mu and -mu for mu = 0..3


def nn_transport(op: Operator, v, path: int):
    """Parallel transport of a [V, 4, 3] field along one path of the network.

    path 0: identity; path 1 + 2*mu: (T v)(x) = s U_mu(x) v(x + mu); path 2 + 2*mu:
    (T v)(x) = s U_mu(x - mu)^+ v(x - mu), with s the same fermion boundary sign as in D.
    Spin is untouched.
    """
    if path == 0:
        return v.copy()
    mu = (path - 1) // 2
    fwd = (path - 1) % 2 == 0
    dims = op.dims
    x = np.indices(dims).reshape(4, -1)
    shift = x.copy()
    shift[mu] = (x[mu] + (1 if fwd else -1)) % dims[mu]
    nbr = ((shift[0] * dims[1] + shift[1]) * dims[2] + shift[2]) * dims[3] + shift[3]
    T = dims[0]
    if fwd:
        U = op.u[:, mu]
        s = np.where((mu == 0) & (x[0] == T - 1), op.bc_t, 1.0)
        out = np.einsum("xij,xsj->xsi", U, v[nbr])
    else:
        U = op.u[nbr, mu]
        s = np.where((mu == 0) & (shift[0] == T - 1), op.bc_t, 1.0)
        out = np.einsum("xji,xsj->xsi", np.conj(U), v[nbr])
    return s[:, None, None] * out


def nn_transport_adj(op: Operator, v, path: int):
    """Adjoint of nn_transport (path +mu and -mu are each other's adjoint)."""
    if path == 0:
        return v.copy()
    mu = (path - 1) // 2
    fwd = (path - 1) % 2 == 0
    return nn_transport(op, v, 2 + 2 * mu if fwd else 1 + 2 * mu)


def nn_layer(op: Operator, W, x):
    """out_a = sum_p sum_b W[p, a, b] (4x4 spin matrix) applied to T_p x_b.

    W: [9, Cout, Cin, 4, 4] complex; x: [Cin, V, 4, 3].
    """
    t = np.stack([np.stack([nn_transport(op, x[b], p) for b in range(x.shape[0])])
                  for p in range(NPATH)])          # [9, Cin, V, 4, 3]
    return np.einsum("pabst,pbxtc->axsc", W, t), t


def nn_forward(op: Operator, weights, r):
    """Network N(r) = L3(L2(L1(r))): linear layers 1 -> 8 -> 8 -> 1 channels.

    Returns the output [V, 4, 3] and the list of layer inputs (for the backward pass).
    """
    x = np.asarray(r, dtype=np.complex128).reshape(1, op.V, 4, 3)
    acts = []
    for W in weights:
        acts.append(x)
        x, _ = nn_layer(op, W, x)
    return x[0], acts


def nn_backward(op: Operator, weights, acts, g_out):
    """Analytic adjoint. g_out = dL/d conj(out) ([V, 4, 3]).

    Returns (grads, g_in): grads[l] = dL/dRe W + i dL/dIm W = 2 dL/d conj(W), and
    g_in = dL/d conj(r).
    """
    g = np.asarray(g_out).reshape(1, op.V, 4, 3)
    grads = [None] * len(weights)
    for l in range(len(weights) - 1, -1, -1):
        W, x = weights[l], acts[l]
        t = np.stack([np.stack([nn_transport(op, x[b], p) for b in range(x.shape[0])])
                      for p in range(NPATH)])
        grads[l] = 2.0 * np.einsum("axsc,pbxtc->pabst", g, np.conj(t))
        gt = np.einsum("pabst,axsc->pbxtc", np.conj(W), g)   # W^+ applied per path
        g = np.stack([sum(nn_transport_adj(op, gt[p, b], p) for p in range(NPATH))
                      for b in range(x.shape[0])])
    return grads, g[0]


def nn_loss(op: Operator, weights, r, e):
    """L = |N(r) - e|^2 / |e|^2 and dL/d conj(out)."""
    out, acts = nn_forward(op, weights, r)
    e = np.asarray(e).reshape(op.V, 4, 3)
    ne2 = _norm(e) ** 2
    d = out - e
    return _norm(d) ** 2 / ne2, d / ne2, acts


def nn_at_sites(dims, bc_t, u, weights, r, sites):
    """N(r) at the listed lexicographic sites only ([n, 4, 3]), for lattices too large for a
    full oracle pass. Layer l's output at x needs its input at x and x +- mu, so the three
    layers are evaluated on the sites within 0, 1, 2 hops of the requested ones, and the
    input is read within 3 hops. Transport as in nn_transport: path 1 + 2 mu is
    s U_mu(x) v(x + mu), path 2 + 2 mu is s U_mu(x - mu)^+ v(x - mu), s = bc_t on hops across
    the time boundary. u: the [V, 4, 3, 3] links; r: the [V, 4, 3] input."""
    dims = tuple(int(d) for d in dims)
    T = dims[0]
    strides = (dims[1] * dims[2] * dims[3], dims[2] * dims[3], dims[3], 1)
    r = np.asarray(r).reshape(-1, 4, 3)

    def coords(lex):
        return [(lex // strides[m]) % dims[m] for m in range(4)]

    def shift(lex, mu, step):
        x = coords(lex)
        y = (x[mu] + step) % dims[mu]
        return lex + (y - x[mu]) * strides[mu]

    def grow(sites_):
        allp = [sites_]
        for mu in range(4):
            allp += [shift(sites_, mu, 1), shift(sites_, mu, -1)]
        return np.unique(np.concatenate(allp))

    out_sites = np.asarray(sites, dtype=np.int64)
    need = [np.unique(out_sites)]
    for _ in range(3):
        need.append(grow(need[-1]))
    # need[3]: input sites, need[2]: layer-1 outputs, need[1]: layer-2, need[0]: layer-3
    x_sites = need[3]
    x = r[x_sites][None]  # [Cin = 1, n, 4, 3]
    for l, W in enumerate(weights):
        o_sites = need[2 - l]
        pos = lambda q: np.searchsorted(x_sites, q)
        t = np.empty((9, x.shape[0], len(o_sites), 4, 3), dtype=np.complex128)
        t[0] = x[:, pos(o_sites)]
        xo = coords(o_sites)
        for mu in range(4):
            fw = shift(o_sites, mu, 1)
            bw = shift(o_sites, mu, -1)
            sf = np.where((mu == 0) & (xo[0] == T - 1), bc_t, 1.0)
            sb = np.where((mu == 0) & (xo[0] == 0), bc_t, 1.0)
            Uf = u[o_sites, mu]
            Ub = np.conj(np.swapaxes(u[bw, mu], -1, -2))
            t[1 + 2 * mu] = sf[None, :, None, None] * np.einsum("nij,bnsj->bnsi", Uf, x[:, pos(fw)])
            t[2 + 2 * mu] = sb[None, :, None, None] * np.einsum("nij,bnsj->bnsi", Ub, x[:, pos(bw)])
        x = np.einsum("pabst,pbntc->ansc", W, t)
        x_sites = o_sites
    return x[0][np.searchsorted(x_sites, out_sites)]


def nn_identity_weights(channels=(1, 8, 8, 1), seed=None, scale=0.0):
    """Weights whose network is the identity map: layer l maps channel 0 to channel 0
    through the identity path with the 4x4 unit spin matrix; optional small noise."""
    rng = np.random.Generator(np.random.PCG64(seed)) if seed is not None else None
    ws = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        W = np.zeros((NPATH, cout, cin, 4, 4), dtype=np.complex128)
        W[0, 0, 0] = np.eye(4)
        if rng is not None and scale:
            W += scale * (rng.standard_normal(W.shape) + 1j * rng.standard_normal(W.shape))
        ws.append(W)
    return ws
