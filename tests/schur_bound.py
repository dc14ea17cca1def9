"""First-order rounding-error bound of the even-odd reduced operator with 16-bit storage.

With storage precision of unit roundoff u, every stored number carries a relative error of
at most u: the input spinor, rows 0 and 1 and the determinant of every link (row 2 is
rebuilt as d conj(row0 x row1): its entries carry at most 3u of the sum of the absolute
values of their two products), the clover blocks A and their inverses, the intermediate
t = A_oo^-1 D_oe psi_e (stored in the output field's odd half) and the output. The FP32
arithmetic in between adds O(2^-24), negligible against u. Propagating these errors through

    stage 1 (odd o):  t = A^-1 h,      h = -1/2 sum_hops P U psi(nbr)
    stage 2 (even e): out = A psi + 1/2 sum_hops P U t(nbr)

entry by entry, with |.| the entrywise absolute value (|P| = |1 -+ gamma_mu| for D and
D^+ alike), gives to first order in u

    dh   <= 1/2 sum |P| (|U| u |psi| + E_U |psi|)
    dt   <= |A^-1| dh + u |A^-1| |h|_abs + u |t|
    dout <= 2u |A| |psi| + 1/2 sum |P| (|U| dt + E_U |t|) + u |out|

where |h|_abs = 1/2 sum |P||U||psi| and E_U is the error matrix of a stored link. The test
compares every component of the GPU result with the oracle's to within this bound (times
1.25 for the second-order terms).
"""
import numpy as np

import oracle


def _abs_hops(op, nb, parity_sites, x, err_u=None):
    """sum over the 8 hops of |P| (x) M x(nbr) at the given sites, M = |U| (err_u None) or
    the link error matrix E_U (err_u = u); x: [V, 4, 3] non-negative."""
    g = oracle.gamma()
    out = np.zeros((len(parity_sites), 4, 3))
    for mu in range(4):
        absP = np.abs(np.eye(4) - g[mu])  # = |1 + gamma_mu| entrywise
        for fwd in (True, False):
            nbr = nb[parity_sites, 2 * mu + (0 if fwd else 1)]
            U = op.u[parity_sites, mu] if fwd else np.conj(np.swapaxes(op.u[nbr, mu], -1, -2))
            if err_u is None:
                M = np.abs(U)
            else:
                M = _link_error(op.u[parity_sites, mu] if fwd else op.u[nbr, mu], err_u)
                if not fwd:
                    M = np.swapaxes(M, -1, -2)
            out += np.einsum("st,nij,ntj->nsi", absP, M, x[nbr])
    return out


def _link_error(U, u):
    """Entrywise error bound of a stored link: rows 0, 1 rounded (u |U|); row 2 rebuilt
    from the rounded rows and the rounded determinant (3u per product, two products)."""
    E = np.empty(U.shape)
    a = np.abs(U)
    E[:, :2] = u * a[:, :2]
    for j in range(3):
        j1, j2 = (j + 1) % 3, (j + 2) % 3
        E[:, 2, j] = 3.0 * u * (a[:, 0, j1] * a[:, 1, j2] + a[:, 0, j2] * a[:, 1, j1])
    return E


def schur_error_bound(op, sc, psi, u, dag=False):
    """Entrywise first-order bound [V, 4, 3] (zero on odd sites) of the error of D^ psi_e
    (or D^+ psi_e) computed with storage unit roundoff u."""
    V = op.V
    nb = oracle.neighbours(op.dims)
    par = oracle.site_parity(op.dims)
    ev, od = np.flatnonzero(par == 0), np.flatnonzero(par == 1)
    psi = np.asarray(psi).reshape(V, 4, 3)
    pe = np.where(sc.even, psi, 0)
    ap = np.abs(pe)
    Aabs = np.abs(op.A)                        # [V, 12, 12]
    Ainv_abs = np.abs(sc.Ainv)
    # exact intermediate and output
    fwd = op.dw_dag if dag else op.dw
    y = fwd(pe)
    t = np.where(sc.odd, sc._ainv(np.where(sc.odd, y, 0)), 0)
    out = (sc.apply_dag if dag else sc.apply)(psi)
    # stage 1 on the odd sites
    h_abs = np.zeros((V, 4, 3))
    h_abs[od] = 0.5 * _abs_hops(op, nb, od, ap)
    dh = np.zeros((V, 4, 3))
    dh[od] = 0.5 * (_abs_hops(op, nb, od, u * ap) + _abs_hops(op, nb, od, ap, err_u=u))
    mat = lambda M, x: np.einsum("nij,nj->ni", M, x.reshape(-1, 12)).reshape(-1, 4, 3)
    dt = np.zeros((V, 4, 3))
    dt[od] = mat(Ainv_abs[od], dh[od]) + u * mat(Ainv_abs[od], h_abs[od]) + u * np.abs(t[od])
    # stage 2 on the even sites
    at = np.abs(t)
    bound = np.zeros((V, 4, 3))
    bound[ev] = (2.0 * u * mat(Aabs[ev], ap[ev])
                 + 0.5 * (_abs_hops(op, nb, ev, dt) + _abs_hops(op, nb, ev, at, err_u=u))
                 + u * np.abs(out[ev]))
    return bound, out
