"""Seeded synthetic inputs: gauge fields, sources and random gauge transformations.

This module holds no arithmetic of the Dirac operator or of the solvers; it only
draws inputs. Both the HIP library (through its Python binding) and the CPU oracle
are fed from here, so the two sides see identical arrays.

Conventions shared by every consumer:

* lattice ``dims = (T, L1, L2, L3)``; direction 0 is time;
* canonical site index ``((x0*L1 + x1)*L2 + x2)*L3 + x3`` (time slowest);
* gauge field: ``su3`` complex128 ``[V, 4, 3, 3]`` (SU(3) part) and ``theta``
  float64 ``[V, 4]`` (U(1) angle); the link is ``U = exp(i*theta) * su3``;
* spinor: complex128 ``[V, 4, 3]`` (spin, colour).

Link recipe: ``V_mu(x) = exp(i*eps*H)`` with ``H`` the traceless Hermitian part of a
3x3 matrix of i.i.d. standard complex Gaussians, computed exactly through an
eigen-decomposition, then re-unitarised (row 1 normalised, row 2 Gram-Schmidt, row 3 =
conj(row1 x row2)) so that the third row is exactly what a 12-real compressed link
rebuilds; ``theta = eps_u1 * a`` with ``a ~ N(0, 1)``. Random numbers come from numpy's
PCG64 with the seed given; the SU(3) draw ``(V, 4, 3, 3, 2)`` comes first, then the
angles ``(V, 4)``.
"""
from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np

# Seeds: gauge field of workload i is 7388 + 10*i (+k for extra ensemble members);
# sources use gauge seed + 1000 + rhs index.
SEED_BASE = 7388


def volume(dims) -> int:
    T, L1, L2, L3 = dims
    return int(T) * int(L1) * int(L2) * int(L3)


def _expm_i_eps_h(h: np.ndarray, eps: float) -> np.ndarray:
    w, q = np.linalg.eigh(h)
    ph = np.exp(1j * eps * w)
    return (q * ph[..., None, :]) @ np.conj(np.swapaxes(q, -1, -2))


def _reunitarise(u: np.ndarray) -> np.ndarray:
    r1 = u[..., 0, :]
    r1 = r1 / np.sqrt(np.sum(np.abs(r1) ** 2, axis=-1, keepdims=True))
    r2 = u[..., 1, :]
    r2 = r2 - np.sum(np.conj(r1) * r2, axis=-1, keepdims=True) * r1
    r2 = r2 / np.sqrt(np.sum(np.abs(r2) ** 2, axis=-1, keepdims=True))
    r3 = np.conj(np.cross(r1, r2))
    return np.stack([r1, r2, r3], axis=-2)


def _su3_from_gauss(g: np.ndarray, eps: float) -> np.ndarray:
    a = g[..., 0] + 1j * g[..., 1]
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[..., None, None] * np.eye(3)
    return _reunitarise(_expm_i_eps_h(h, eps))


def gauge_field(dims, eps: float = 0.3, eps_u1: float = 0.1, seed: int = SEED_BASE,
                threads: int | None = None):
    """Return ``(su3, theta)`` for the near-identity SU(3) x U(1) recipe above."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((V, 4, 3, 3, 2))
    a = rng.standard_normal((V, 4))
    su3 = np.empty((V, 4, 3, 3), dtype=np.complex128)
    n = V * 4
    gf = g.reshape(n, 3, 3, 2)
    out = su3.reshape(n, 3, 3)
    chunk = 1 << 16
    starts = list(range(0, n, chunk))
    nthr = threads or min(16, os.cpu_count() or 1)

    def work(s):
        e = min(n, s + chunk)
        out[s:e] = _su3_from_gauss(gf[s:e], eps)

    if len(starts) > 1 and nthr > 1:
        with _cf.ThreadPoolExecutor(nthr) as ex:
            list(ex.map(work, starts))
    else:
        for s in starts:
            work(s)
    theta = eps_u1 * a
    return su3, theta


def unit_gauge_field(dims):
    V = volume(dims)
    su3 = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    su3[..., 0, 0] = su3[..., 1, 1] = su3[..., 2, 2] = 1.0
    return su3, np.zeros((V, 4))


def abelian_flux_theta(dims, n_flux: int, plane=(1, 2)):
    """U(1) angles of a constant field strength in the (mu, nu) plane of a periodic torus.

    Every plaquette in that plane equals exp(i*phi) with phi = 2*pi*n_flux/(L_mu*L_nu);
    all other plaquettes are 1. Construction: U_nu(x) = exp(i*phi*x_mu), and
    U_mu(x) = exp(-i*phi*L_mu*x_nu) on the last slice x_mu = L_mu - 1, else 1.
    """
    mu, nu = plane
    T, L1, L2, L3 = dims
    L = dims
    phi = 2.0 * np.pi * n_flux / (L[mu] * L[nu])
    x = np.indices((T, L1, L2, L3)).reshape(4, -1)
    theta = np.zeros((volume(dims), 4))
    theta[:, nu] = phi * x[mu]
    last = x[mu] == L[mu] - 1
    theta[last, mu] = -phi * L[mu] * x[nu][last]
    return theta, phi


def gaussian_spinor(dims, seed: int) -> np.ndarray:
    """Complex Gaussian spinor, Re and Im ~ N(0, 1), shape [V, 4, 3]."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((V, 4, 3, 2))
    return g[..., 0] + 1j * g[..., 1]


def point_spinor(dims, spin: int, colour: int, site: int = 0) -> np.ndarray:
    V = volume(dims)
    s = np.zeros((V, 4, 3), dtype=np.complex128)
    s[site, spin, colour] = 1.0
    return s


def plane_wave(dims, p, u) -> np.ndarray:
    """psi(x) = exp(i p.x) u, u a [4, 3] complex amplitude."""
    x = np.indices(tuple(dims)).reshape(4, -1).T.astype(np.float64)
    ph = np.exp(1j * (x @ np.asarray(p, dtype=np.float64)))
    return ph[:, None, None] * np.asarray(u)[None]


def random_gauge_transform(dims, seed: int) -> np.ndarray:
    """G(x) in SU(3) x U(1), shape [V, 3, 3]."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((V, 3, 3, 2))
    a = rng.standard_normal(V)
    su3 = _su3_from_gauss(g, 1.0)
    return np.exp(1j * a)[:, None, None] * su3
