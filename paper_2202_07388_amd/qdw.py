"""Python binding of libqdw (ctypes). Argument marshalling only: every step of the
operator and the solvers runs in the HIP kernels of ``libqdw.so``.

PyTorch supplies device memory and the current stream; fields are plain byte tensors
holding the library's eo-SoA layout. The binding fails loudly when the library is
missing or when no GPU is present: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqdw.so")

PREC = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
REAL_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}

# machine epsilon 2^-m of the storage formats (paper Table 1)
EPS = {"f64": 2.0 ** -52, "f32": 2.0 ** -23, "f16": 2.0 ** -10, "bf16": 2.0 ** -7}


class QdwError(RuntimeError):
    pass


class Lattice(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int), ("L1", ctypes.c_int), ("L2", ctypes.c_int),
                ("L3", ctypes.c_int), ("bc_t", ctypes.c_int)]


_lib = None
_P = ctypes.c_void_p


def load():
    """Load libqdw.so and declare argument types of every exported entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise QdwError("libqdw.so is not built (run __graft_entry__.build() or "
                       "python -m paper_2202_07388_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    L.qdw_last_error.restype = ctypes.c_char_p
    L.qdw_op_device_bytes.argtypes = [ctypes.POINTER(Lattice)]
    L.qdw_op_device_bytes.restype = ctypes.c_size_t
    L.qdw_op_host_bytes.argtypes = []
    L.qdw_op_host_bytes.restype = ctypes.c_size_t
    L.qdw_create.argtypes = [ctypes.POINTER(Lattice), _P, _P, ctypes.c_double,
                             ctypes.c_double, _P, ctypes.c_size_t, _P, ctypes.c_size_t, _P,
                             ctypes.POINTER(_P)]
    L.qdw_destroy.argtypes = [_P]
    L.qdw_volume.argtypes = [_P]
    L.qdw_volume.restype = ctypes.c_long
    L.qdw_field_bytes.argtypes = [_P, ctypes.c_int]
    L.qdw_field_bytes.restype = ctypes.c_size_t
    for f in (L.qdw_pack, L.qdw_unpack):
        f.argtypes = [_P, _P, _P, ctypes.c_int, _P]
    for f in (L.dw_apply, L.dw_dag_apply):
        f.argtypes = [_P, _P, _P, ctypes.c_int, _P]
    for name in ("dw_schur_apply", "dw_schur_dag_apply"):
        if hasattr(L, name):
            getattr(L, name).argtypes = [_P, _P, _P, ctypes.c_int, _P]
    _declare_solvers(L)
    _lib = L
    return L


def _declare_solvers(L):
    """Solver entry points are declared when the library exports them."""
    for name, args, res in _OPTIONAL:
        if hasattr(L, name):
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("nreset", ctypes.c_int), ("n_dw_hi", ctypes.c_int),
                ("n_dw_lo", ctypes.c_int), ("n_steps", ctypes.c_int),
                ("rel_res_true", ctypes.c_double), ("t_sec", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CgneParams(ctypes.Structure):
    _fields_ = [("res", ctypes.c_double), ("nmx", ctypes.c_int), ("inner", ctypes.c_int),
                ("delta", ctypes.c_double), ("keep_p", ctypes.c_int), ("cascade", ctypes.c_int),
                ("cascade_c", ctypes.c_double), ("schur", ctypes.c_int)]


class SapGcrParams(ctypes.Structure):
    _fields_ = [("res", ctypes.c_double), ("nmx", ctypes.c_int), ("nkv", ctypes.c_int),
                ("ncy", ctypes.c_int), ("nmr", ctypes.c_int), ("bs", ctypes.c_int * 4),
                ("sdtype", ctypes.c_int), ("precond", ctypes.c_int),
                ("nn_weights", ctypes.c_void_p), ("sap_alpha", ctypes.c_double)]


PRECOND = {"none": 0, "sap": 1, "nn": 2, "nn_sap": 3, "sap_adaptive": 4, "sap_eo": 5}

_OPTIONAL: list = [
    ("qdw_sap_gcr_workspace_bytes", [_P, ctypes.POINTER(SapGcrParams)], ctypes.c_size_t),
    ("sap_gcr_solve", [_P, _P, _P, ctypes.POINTER(SapGcrParams), _P, ctypes.c_size_t,
                       ctypes.POINTER(Info), _P], ctypes.c_int),
    ("qdw_sap_workspace_bytes", [_P, ctypes.c_int], ctypes.c_size_t),
    ("sap_adaptive_apply", [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                            ctypes.c_double, ctypes.POINTER(ctypes.c_int * 4), ctypes.c_int, _P,
                            ctypes.c_size_t, ctypes.POINTER(ctypes.c_int), _P, _P], ctypes.c_int),
    ("sap_apply", [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int * 4),
                   ctypes.c_int, _P, ctypes.c_size_t, _P], ctypes.c_int),
    ("sap_eo_apply", [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int * 4),
                      ctypes.c_int, _P, ctypes.c_size_t, _P], ctypes.c_int),
    ("qdw_sap_noalloc_max_bytes", [], ctypes.c_size_t),
    ("qdw_full_links_bytes", [_P], ctypes.c_size_t),
    ("qdw_set_full_links", [_P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    ("dw_apply_full_links", [_P, _P, _P, ctypes.c_int, _P], ctypes.c_int),
    ("sap_apply_noalloc", [_P, _P, _P, ctypes.c_int, ctypes.c_int,
                           ctypes.POINTER(ctypes.c_int * 4), ctypes.c_int, _P], ctypes.c_int),
    ("qdw_axpby", [_P, ctypes.c_double, _P, ctypes.c_double, _P, ctypes.c_int, _P], ctypes.c_int),
    ("qdw_norm2", [_P, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _P], ctypes.c_int),
    ("qdw_cdot", [_P, _P, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_double * 2), _P],
     ctypes.c_int),
    ("qdw_convert", [_P, _P, ctypes.c_int, _P, ctypes.c_int, ctypes.c_double, _P],
     ctypes.c_int),
    ("qdw_nn_weight_count", [], ctypes.c_int),
    ("qdw_nn_workspace_bytes", [_P, ctypes.c_int], ctypes.c_size_t),
    ("nn_forward", [_P, _P, _P, _P, ctypes.c_int, _P, ctypes.c_size_t, _P], ctypes.c_int),
    ("nn_backward", [_P, _P, _P, _P, _P, _P, ctypes.c_int, _P, ctypes.c_size_t, _P],
     ctypes.c_int),
    ("nn_train_step", [_P, _P, _P, ctypes.c_int, ctypes.c_double, _P, _P, ctypes.c_int,
                       ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _P,
                       ctypes.c_size_t, _P], ctypes.c_int),
    ("dw_apply_multi", [_P, _P, _P, ctypes.c_int, ctypes.c_int, _P], ctypes.c_int),
    ("qdw_autotune_workspace_bytes", [_P, ctypes.c_int, ctypes.c_int], ctypes.c_size_t),
    ("qdw_autotune", [_P, ctypes.c_int, ctypes.c_int, _P, ctypes.c_size_t, ctypes.c_char_p,
                      ctypes.c_size_t, _P], ctypes.c_int),
    ("qdw_set_dw_shape", [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int, ctypes.c_int], ctypes.c_int),
    ("qdw_get_dw_shape", [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int * 5)], ctypes.c_int),
    ("qdw_sap_gcr_batched_workspace_bytes", [_P, ctypes.c_int, ctypes.POINTER(SapGcrParams)],
     ctypes.c_size_t),
    ("sap_gcr_solve_batched", [_P, _P, _P, ctypes.c_int, ctypes.POINTER(SapGcrParams), _P,
                               ctypes.c_size_t, _P, ctypes.POINTER(ctypes.c_double), _P],
     ctypes.c_int),
    ("qdw_batch_create", [_P, ctypes.c_int, ctypes.POINTER(SapGcrParams), ctypes.c_int, _P,
                          ctypes.c_size_t, ctypes.POINTER(_P)], ctypes.c_int),
    ("qdw_batch_solve", [_P, _P, _P, _P, ctypes.POINTER(ctypes.c_int), _P], ctypes.c_int),
    ("qdw_batch_capture_ms", [_P], ctypes.c_double),
    ("qdw_batch_destroy", [_P], ctypes.c_int),
    ("qdw_cgne_workspace_bytes", [_P, ctypes.POINTER(CgneParams)], ctypes.c_size_t),
    ("cgne_solve", [_P, _P, _P, ctypes.POINTER(CgneParams), _P, ctypes.c_size_t,
                    ctypes.POINTER(Info), _P], ctypes.c_int),
]


def _check(rc: int, what: str):
    if rc != 0:
        msg = load().qdw_last_error().decode(errors="replace")
        raise QdwError("%s failed (code %d): %s" % (what, rc, msg))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise QdwError("libqdw needs a HIP GPU; none is visible")
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    if not t.is_cuda:
        raise QdwError("expected a device tensor")
    if not t.is_contiguous():
        raise QdwError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


class Op:
    """A Wilson-clover operator resident on the current GPU (qdw_create)."""

    def __init__(self, dims, su3, theta, m0: float, csw: float, bc_t: int = -1):
        torch = _torch()
        L = load()
        self.dims = tuple(int(v) for v in dims)
        self.V = int(np.prod(self.dims))
        self.m0, self.csw, self.bc_t = float(m0), float(csw), int(bc_t)
        dev = torch.device("cuda", torch.cuda.current_device())
        su3_t = torch.as_tensor(np.ascontiguousarray(su3, dtype=np.complex128)
                                if isinstance(su3, np.ndarray) else su3)
        th_t = torch.as_tensor(np.ascontiguousarray(theta, dtype=np.float64)
                               if isinstance(theta, np.ndarray) else theta)
        su3_d = torch.view_as_real(su3_t.to(dev).contiguous()).contiguous()
        th_d = th_t.to(dev, dtype=torch.float64).contiguous()
        if su3_d.numel() != self.V * 4 * 9 * 2 or th_d.numel() != self.V * 4:
            raise QdwError("gauge field shape does not match the lattice")
        lat = Lattice(*self.dims, self.bc_t)
        nd = int(L.qdw_op_device_bytes(ctypes.byref(lat)))
        if nd == 0:
            raise QdwError("qdw_create: %s" % L.qdw_last_error().decode(errors="replace"))
        # the operator's device and host blocks are torch tensors: PyTorch owns the memory
        self._dev_mem = torch.empty(nd, dtype=torch.uint8, device=dev)
        self._host_mem = torch.empty(int(L.qdw_op_host_bytes()), dtype=torch.uint8,
                                     pin_memory=True)
        h = _P()
        _check(L.qdw_create(ctypes.byref(lat), _ptr(su3_d), _ptr(th_d), self.m0, self.csw,
                            _ptr(self._dev_mem), nd, ctypes.c_void_p(self._host_mem.data_ptr()),
                            self._host_mem.numel(), _stream(), ctypes.byref(h)), "qdw_create")
        self._h = h
        self.device = dev

    @property
    def handle(self):
        return self._h

    @property
    def device_bytes(self) -> int:
        """Bytes of the caller-owned device block the operator lives in."""
        return self._dev_mem.numel()

    def close(self):
        if getattr(self, "_h", None):
            load().qdw_destroy(self._h)
            self._h = None
        self._dev_mem = None
        self._host_mem = None
        self._full_links = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def field_bytes(self, prec: str = "f64") -> int:
        return int(load().qdw_field_bytes(self._h, PREC[prec]))

    def new_field(self, prec: str = "f64", zero: bool = True):
        torch = _torch()
        n = self.field_bytes(prec)
        t = torch.zeros(n, dtype=torch.uint8, device=self.device) if zero else \
            torch.empty(n, dtype=torch.uint8, device=self.device)
        return t

    def pack(self, canonical, prec: str = "f64", out=None):
        """canonical complex128 [V, 4, 3] (numpy or tensor) -> eo-SoA byte tensor."""
        torch = _torch()
        c = torch.as_tensor(canonical).to(self.device, dtype=torch.complex128).contiguous()
        if c.numel() != self.V * 12:
            raise QdwError("spinor shape does not match the lattice")
        out = self.new_field(prec) if out is None else out
        _check(load().qdw_pack(self._h, _ptr(torch.view_as_real(c)), _ptr(out), PREC[prec],
                               _stream()), "qdw_pack")
        return out

    def unpack(self, eo, prec: str = "f64"):
        """eo-SoA byte tensor -> canonical complex128 [V, 4, 3] device tensor."""
        torch = _torch()
        out = torch.empty((self.V, 4, 3, 2), dtype=torch.float64, device=self.device)
        _check(load().qdw_unpack(self._h, _ptr(eo), _ptr(out), PREC[prec], _stream()),
               "qdw_unpack")
        return torch.view_as_complex(out)


def dw_apply(op: Op, x, out, prec: str = "f64"):
    _check(load().dw_apply(op.handle, _ptr(x), _ptr(out), PREC[prec], _stream()), "dw_apply")
    return out


def dw_dag_apply(op: Op, x, out, prec: str = "f64"):
    _check(load().dw_dag_apply(op.handle, _ptr(x), _ptr(out), PREC[prec], _stream()),
           "dw_dag_apply")
    return out


def dw_schur_apply(op: Op, x, out, prec: str = "f64"):
    """Even half of out = D^ (even half of x); the odd half of out is scratch."""
    _check(load().dw_schur_apply(op.handle, _ptr(x), _ptr(out), PREC[prec], _stream()),
           "dw_schur_apply")
    return out


def dw_schur_dag_apply(op: Op, x, out, prec: str = "f64"):
    _check(load().dw_schur_dag_apply(op.handle, _ptr(x), _ptr(out), PREC[prec], _stream()),
           "dw_schur_dag_apply")
    return out


def axpby(op: Op, a: float, x, b: float, y, prec: str = "f64"):
    """y = a x + b y."""
    _check(load().qdw_axpby(op.handle, a, _ptr(x), b, _ptr(y), PREC[prec], _stream()),
           "qdw_axpby")
    return y


def norm2(op: Op, x, prec: str = "f64") -> float:
    out = ctypes.c_double()
    _check(load().qdw_norm2(op.handle, _ptr(x), PREC[prec], ctypes.byref(out), _stream()),
           "qdw_norm2")
    return out.value


def cdot(op: Op, x, y, prec: str = "f64") -> complex:
    out = (ctypes.c_double * 2)()
    _check(load().qdw_cdot(op.handle, _ptr(x), _ptr(y), PREC[prec], ctypes.byref(out),
                           _stream()), "qdw_cdot")
    return complex(out[0], out[1])


def convert(op: Op, x, px: str, y, py: str, s: float = 1.0):
    """y = s x, from precision px to py."""
    _check(load().qdw_convert(op.handle, _ptr(x), PREC[px], _ptr(y), PREC[py], s, _stream()),
           "qdw_convert")
    return y


def _workspace(op: Op, nbytes: int):
    """Device workspace owned by the Python Op (grown on demand, reused across calls)."""
    torch = _torch()
    ws = getattr(op, "_ws", None)
    if ws is None or ws.numel() < nbytes:
        op._ws = None
        op._ws = torch.empty(nbytes, dtype=torch.uint8, device=op.device)
    return op._ws


def cgne_solve(op: Op, eta, psi, res: float = 1e-10, nmx: int = 20000, inner: str = "f64",
               delta: float = -1.0, keep_p: bool = True, cascade: bool = False,
               cascade_c: float = 0.0, schur: bool = False) -> dict:
    """Solve D^+ D psi = eta (FP64 eo-SoA fields) with the normal-equation CG; cascade=True
    runs the BF16 -> FP32 -> FP64 precision cascade (inner is then ignored); schur=True
    solves the even-odd reduced system D^+ D^ psi_e = eta_e on the even halves."""
    L = load()
    prm = CgneParams(res, nmx, PREC[inner], delta, 1 if keep_p else 0, 1 if cascade else 0,
                     cascade_c, 1 if schur else 0)
    nb = int(L.qdw_cgne_workspace_bytes(op.handle, ctypes.byref(prm)))
    ws = _workspace(op, nb)
    info = Info()
    _check(L.cgne_solve(op.handle, _ptr(eta), _ptr(psi), ctypes.byref(prm), _ptr(ws),
                        ws.numel(), ctypes.byref(info), _stream()), "cgne_solve")
    return info.as_dict()


def sap_gcr_solve(op: Op, eta, psi, res: float = 1e-10, nmx: int = 2000, nkv: int = 16,
                  ncy: int = 5, nmr: int = 4, bs=(4, 4, 4, 4), sdtype: str = "f16",
                  precond: str = "sap", nn_weights=None, alpha: float = 0.9) -> dict:
    """Solve D psi = eta (FP64 eo-SoA fields) with (SAP-preconditioned) flexible GCR.
    precond "sap_adaptive": ncy and nmr are maxima, alpha the MR exit factor."""
    L = load()
    w = ctypes.c_void_p(nn_weights.data_ptr()) if nn_weights is not None else None
    prm = SapGcrParams(res, nmx, nkv, ncy, nmr, (ctypes.c_int * 4)(*bs), PREC[sdtype],
                       PRECOND[precond], w, alpha)
    nb = int(L.qdw_sap_gcr_workspace_bytes(op.handle, ctypes.byref(prm)))
    if nb == 0:
        raise QdwError("bad SAP-GCR settings")
    ws = _workspace(op, nb)
    info = Info()
    _check(L.sap_gcr_solve(op.handle, _ptr(eta), _ptr(psi), ctypes.byref(prm), _ptr(ws),
                           ws.numel(), ctypes.byref(info), _stream()), "sap_gcr_solve")
    return info.as_dict()


def solve_from(op: Op, eta, x0, psi, solver: str = "gcr", res: float = 1e-10, **kw) -> dict:
    """Warm start: solve D psi = eta ("gcr", settings as sap_gcr_solve) or D^+ D psi = eta
    ("cgne", settings as cgne_solve) from the guess x0 (FP64 fields; x0 is not changed).
    The solver runs on the residual system A delta = r0 = eta - A x0 to the same absolute
    target, res |eta| / |r0|, and psi = x0 + delta; rel_res_true is then recomputed for psi
    against eta. Every step runs in the library's kernels."""
    if solver not in ("gcr", "cgne"):
        raise QdwError("solve_from: solver 'gcr' or 'cgne'")
    t = op.new_field("f64") if solver == "cgne" else None

    def apply(x, out):
        if solver == "gcr":
            dw_apply(op, x, out, "f64")
        else:
            dw_apply(op, x, t, "f64")
            dw_dag_apply(op, t, out, "f64")

    r0 = op.new_field("f64")
    apply(x0, r0)
    axpby(op, 1.0, eta, -1.0, r0)                      # r0 = eta - A x0
    n_eta, n_r0 = np.sqrt(norm2(op, eta)), np.sqrt(norm2(op, r0))
    if not (n_eta > 0.0):
        raise QdwError("solve_from: zero source")
    if n_r0 <= res * n_eta:                             # the guess already meets the target
        axpby(op, 1.0, x0, 0.0, psi)
        return {"status": 0, "nreset": 0, "n_dw_hi": 1, "n_dw_lo": 0, "n_steps": 0,
                "rel_res_true": float(n_r0 / n_eta), "t_sec": 0.0}
    rel = res * n_eta / n_r0
    info = (sap_gcr_solve(op, r0, psi, res=rel, **kw) if solver == "gcr"
            else cgne_solve(op, r0, psi, res=rel, **kw))
    axpby(op, 1.0, x0, 1.0, psi)                        # psi = x0 + delta
    apply(psi, r0)
    axpby(op, 1.0, eta, -1.0, r0)
    info["rel_res_true"] = float(np.sqrt(norm2(op, r0)) / n_eta)
    return info


def _ptr_array(ts):
    return (ctypes.c_void_p * len(ts))(*[_ptr(t).value for t in ts])


def dw_apply_multi(op: Op, xs, outs, prec: str = "f64"):
    """outs[r] = D xs[r] for every r, in one launch."""
    if len(xs) != len(outs):
        raise QdwError("dw_apply_multi: as many outputs as inputs")
    _check(load().dw_apply_multi(op.handle, _ptr_array(xs), _ptr_array(outs), len(xs),
                                 PREC[prec], _stream()), "dw_apply_multi")
    return outs


def autotune(op: Op, prec: str = "f64", nrhs: int = 1) -> str:
    """Pick the fastest D-kernel shape for this operator; returns the tuner's report."""
    torch = _torch()
    L = load()
    nb = int(L.qdw_autotune_workspace_bytes(op.handle, PREC[prec], nrhs))
    if nb == 0:
        raise QdwError("qdw_autotune: bad arguments")
    work = torch.empty(nb, dtype=torch.uint8, device=op.device)
    buf = ctypes.create_string_buffer(4096)
    _check(L.qdw_autotune(op.handle, PREC[prec], nrhs, _ptr(work), nb, buf, len(buf), _stream()),
           "qdw_autotune")
    del work
    return buf.value.decode()


# ------------------------------------------------------------------ autotune cache
#
# The tuner times every candidate shape (tens of milliseconds at 32^3 x 64); its choice
# depends on the lattice, the precision, the number of fields per launch, the device and the
# D kernels themselves, so a cache entry is keyed by all five and a kernel source change
# misses the cache.

_TUNE_SOURCES = ("dirac.hip", "dirac_core.h", "qdw_internal.h")


def kernel_version() -> str:
    """A short hash of the D kernels' sources next to the library (empty if absent)."""
    import hashlib
    h = hashlib.sha256()
    for name in _TUNE_SOURCES:
        f = os.path.join(_HERE, "csrc", name)
        if not os.path.exists(f):
            return ""
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def tune_key(dims, prec: str, nrhs: int, device: str, kernels: str) -> str:
    return "%s|%s|nrhs%d|%s|%s" % ("x".join(str(int(v)) for v in dims), prec, int(nrhs),
                                   device, kernels)


def read_tune_cache(path: str, key: str):
    """The cached (ts, nt, pipe, walk, march) for key, or None (no file, no entry, or an
    entry that is not five integers)."""
    import json
    try:
        with open(path) as fh:
            entries = json.load(fh).get("entries", {})
    except (OSError, ValueError, AttributeError):
        return None
    shape = entries.get(key) if isinstance(entries, dict) else None
    if isinstance(shape, list) and len(shape) == 5 and all(isinstance(v, int) for v in shape):
        return tuple(shape)
    return None


def write_tune_cache(path: str, key: str, shape) -> None:
    """Add or replace one entry; the file is rewritten whole through a temporary file, so
    a reader never sees a partial file; an entry that another process writes between this
    call's read and its write is lost."""
    import json
    data = {"version": 1, "entries": {}}
    try:
        with open(path) as fh:
            old = json.load(fh)
        if isinstance(old, dict) and isinstance(old.get("entries"), dict):
            data["entries"] = old["entries"]
    except (OSError, ValueError):
        pass
    data["entries"][key] = [int(v) for v in shape]
    tmp = "%s.tmp%d" % (path, os.getpid())
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune_cached(op: Op, prec: str = "f64", nrhs: int = 1, path: str | None = None):
    """Set the D-kernel shape for this operator from the cache file when it holds one for
    this lattice, precision, field count, device and kernel version; otherwise run the
    tuner and store its choice. Returns ("cached" or "tuned", shape)."""
    torch = _torch()
    path = path or os.path.join(_HERE, "dw_shapes.json")
    key = tune_key(op.dims, prec, nrhs, torch.cuda.get_device_name(op.device), kernel_version())
    shape = read_tune_cache(path, key)
    if shape is not None:
        set_dw_shape(op, prec, *shape)
        return "cached", shape
    autotune(op, prec, nrhs)
    shape = get_dw_shape(op, prec)
    write_tune_cache(path, key, shape)
    return "tuned", shape


def set_dw_shape(op: Op, prec: str, ts: int, nt: int, pipe: int, walk: int = 0, march: int = 0):
    """Pin the D kernel's shape for one precision (what the autotuner would choose)."""
    _check(load().qdw_set_dw_shape(op.handle, PREC[prec], ts, nt, pipe, walk, march),
           "qdw_set_dw_shape")


def get_dw_shape(op: Op, prec: str = "f64"):
    """(ts, nt, pipe, walk, march) of the D kernel for one precision."""
    out = (ctypes.c_int * 5)()
    _check(load().qdw_get_dw_shape(op.handle, PREC[prec], ctypes.byref(out)), "qdw_get_dw_shape")
    return tuple(out)


def sap_gcr_solve_batched(ops, etas, psis, res: float = 1e-10, nmx: int = 2000, nkv: int = 16,
                          ncy: int = 5, nmr: int = 4, bs=(4, 4, 4, 4), sdtype: str = "f16",
                          precond: str = "sap", work=None):
    """Solve D_j psi_j = eta_j for every j together (ops may repeat and differ in volume);
    returns (list of per-solve result dicts, graph set-up time in ms)."""
    L = load()
    torch = _torch()
    n = len(ops)
    if not (len(etas) == n and len(psis) == n):
        raise QdwError("sap_gcr_solve_batched: one source and one solution per operator")
    prm = SapGcrParams(res, nmx, nkv, ncy, nmr, (ctypes.c_int * 4)(*bs), PREC[sdtype],
                       PRECOND[precond], None, 0.9)
    hs = (ctypes.c_void_p * n)(*[o.handle for o in ops])
    nb = int(L.qdw_sap_gcr_batched_workspace_bytes(hs, n, ctypes.byref(prm)))
    if nb == 0:
        raise QdwError("bad batched SAP-GCR settings")
    if work is None or work.numel() < nb:
        work = torch.empty(nb, dtype=torch.uint8, device=ops[0].device)
    infos = (Info * n)()
    gms = ctypes.c_double(0.0)
    _check(L.sap_gcr_solve_batched(hs, _ptr_array(etas), _ptr_array(psis), n, ctypes.byref(prm),
                                   _ptr(work), work.numel(), infos, ctypes.byref(gms),
                                   _stream()), "sap_gcr_solve_batched")
    return [i.as_dict() for i in infos], gms.value


class Batch:
    """A captured batch of flexible-GCR solves (qdw_batch): the graph of `cycles` restart
    cycles is built once over the operators `ops` (which may repeat and differ in volume)
    and replayed by every solve; the workspace is a torch tensor owned by the plan."""

    def __init__(self, ops, res: float = 1e-10, nmx: int = 2000, nkv: int = 16, ncy: int = 5,
                 nmr: int = 4, bs=(4, 4, 4, 4), sdtype: str = "f16", precond: str = "sap",
                 cycles: int = 1):
        L = load()
        torch = _torch()
        self.ops = list(ops)
        self.n = len(self.ops)
        self._prm = SapGcrParams(res, nmx, nkv, ncy, nmr, (ctypes.c_int * 4)(*bs), PREC[sdtype],
                                 PRECOND[precond], None, 0.9)
        self._hs = (ctypes.c_void_p * self.n)(*[o.handle for o in self.ops])
        nb = int(L.qdw_sap_gcr_batched_workspace_bytes(self._hs, self.n, ctypes.byref(self._prm)))
        if nb == 0:
            raise QdwError("bad batched SAP-GCR settings")
        self.work = torch.empty(nb, dtype=torch.uint8, device=self.ops[0].device)
        h = _P()
        _check(L.qdw_batch_create(self._hs, self.n, ctypes.byref(self._prm), cycles,
                                  _ptr(self.work), nb, ctypes.byref(h)), "qdw_batch_create")
        self._h = h
        self.cycles = cycles
        self.capture_ms = float(L.qdw_batch_capture_ms(h))

    def solve(self, etas, psis):
        """Solve every problem; returns (per-solve result dicts, graph launches)."""
        if not (len(etas) == self.n and len(psis) == self.n):
            raise QdwError("Batch.solve: one source and one solution per operator")
        infos = (Info * self.n)()
        nl = ctypes.c_int(0)
        _check(load().qdw_batch_solve(self._h, _ptr_array(etas), _ptr_array(psis), infos,
                                      ctypes.byref(nl), _stream()), "qdw_batch_solve")
        return [i.as_dict() for i in infos], nl.value

    def close(self):
        if getattr(self, "_h", None):
            load().qdw_batch_destroy(self._h)
            self._h = None
        self.work = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sap_adaptive_apply(op: Op, rho, phi, ncy_max: int = 20, nmr_max: int = 20,
                       alpha: float = 0.9, tol: float = 0.0, bs=(4, 4, 4, 4),
                       sdtype: str = "f16", steps=None) -> int:
    """phi = adaptive SAP applied to rho (FP64 fields); returns the cycles run. steps: an
    optional device int32 tensor of ncy_max * 2 * (blocks / 2) entries for the per-block MR
    step counts."""
    L = load()
    nb = int(L.qdw_sap_workspace_bytes(op.handle, PREC[sdtype]))
    ws = _workspace(op, nb)
    cyc = ctypes.c_int(0)
    sp = _ptr(steps) if steps is not None else None
    _check(L.sap_adaptive_apply(op.handle, _ptr(rho), _ptr(phi), ncy_max, nmr_max, alpha, tol,
                                ctypes.byref((ctypes.c_int * 4)(*bs)), PREC[sdtype], _ptr(ws),
                                ws.numel(), ctypes.byref(cyc), sp, _stream()),
           "sap_adaptive_apply")
    return cyc.value


def sap_apply(op: Op, rho, phi, ncy: int = 5, nmr: int = 4, bs=(4, 4, 4, 4),
              sdtype: str = "f16", eo: bool = False):
    """phi = M_SAP rho (FP64 eo-SoA fields); eo=True solves the blocks through their
    even-odd reduction (sap_eo_apply)."""
    L = load()
    nb = int(L.qdw_sap_workspace_bytes(op.handle, PREC[sdtype]))
    if nb == 0:
        raise QdwError("bad SAP storage precision")
    ws = _workspace(op, nb)
    b = (ctypes.c_int * 4)(*bs)
    fn, name = (L.sap_eo_apply, "sap_eo_apply") if eo else (L.sap_apply, "sap_apply")
    _check(fn(op.handle, _ptr(rho), _ptr(phi), ncy, nmr, ctypes.byref(b), PREC[sdtype],
              _ptr(ws), ws.numel(), _stream()), name)
    return phi


def set_full_links(op: Op):
    """Form op's FP64 links as full 3x3 matrices (the uncompressed control) in a device
    block taken from torch and kept on op."""
    torch = _torch()
    n = int(load().qdw_full_links_bytes(op.handle))
    op._full_links = torch.empty(n, dtype=torch.uint8, device=op.device)
    _check(load().qdw_set_full_links(op.handle, _ptr(op._full_links), n, _stream()),
           "qdw_set_full_links")


def dw_apply_full_links(op: Op, x, y, dagger: bool = False):
    """y = D x (D^+ x) in FP64 with the full-matrix links of set_full_links."""
    _check(load().dw_apply_full_links(op.handle, _ptr(x), _ptr(y), int(dagger), _stream()),
           "dw_apply_full_links")
    return y


def sap_apply_noalloc(op: Op, rho, phi, ncy: int = 5, nmr: int = 4, bs=(4, 4, 4, 4),
                      sdtype: str = "f16"):
    """phi = M_SAP rho with the library's static device scratch: no workspace, no
    allocation (lattices whose SAP fields fit qdw_sap_noalloc_max_bytes())."""
    b = (ctypes.c_int * 4)(*bs)
    _check(load().sap_apply_noalloc(op.handle, _ptr(rho), _ptr(phi), ncy, nmr, ctypes.byref(b),
                                    PREC[sdtype], _stream()), "sap_apply_noalloc")
    return phi


# ---------------------------------------------------------------- learned preconditioner

NN_CHANNELS = (1, 8, 8, 1)
NN_PATHS = 9


def nn_weight_count() -> int:
    return int(load().qdw_nn_weight_count())


def nn_weights_tensor(layers):
    """Flatten per-layer complex weights [9, Cout, Cin, 4, 4] into the library's FP32
    interleaved layout on the current device."""
    torch = _torch()
    flat = np.concatenate([np.asarray(w, dtype=np.complex128).reshape(-1) for w in layers])
    if flat.size != nn_weight_count():
        raise QdwError("weights do not match the 1-8-8-1 network")
    re_im = np.stack([flat.real, flat.imag], axis=-1).astype(np.float32).reshape(-1)
    return torch.as_tensor(re_im).to(torch.device("cuda", torch.cuda.current_device()))


def nn_weights_layers(t):
    """Inverse of nn_weights_tensor: list of complex numpy arrays [9, Cout, Cin, 4, 4]."""
    a = t.detach().cpu().numpy().astype(np.float64).reshape(-1, 2)
    z = a[:, 0] + 1j * a[:, 1]
    out, o = [], 0
    for cin, cout in zip(NN_CHANNELS[:-1], NN_CHANNELS[1:]):
        n = NN_PATHS * cout * cin * 16
        out.append(z[o:o + n].reshape(NN_PATHS, cout, cin, 4, 4))
        o += n
    return out


def _nn_ws(op: Op, training: bool, extra: int = 0):
    torch = _torch()
    nb = int(load().qdw_nn_workspace_bytes(op.handle, 1 if training else 0)) + extra
    attr = "_nnws_t" if training else "_nnws_f"
    ws = getattr(op, attr, None)
    if ws is None or ws.numel() < nb:
        setattr(op, attr, None)
        ws = torch.empty(nb, dtype=torch.uint8, device=op.device)
        setattr(op, attr, ws)
    return ws


def nn_forward(op: Op, weights, x, out, f32_mixing: bool = False):
    """out = N(x) for FP64 eo-SoA fields."""
    ws = _nn_ws(op, False)
    _check(load().nn_forward(op.handle, _ptr(weights), _ptr(x), _ptr(out),
                             1 if f32_mixing else 0, _ptr(ws), ws.numel(), _stream()),
           "nn_forward")
    return out


def nn_backward(op: Op, weights, x, gout, dW, gin, f32_mixing: bool = False):
    """Real gradients: dW and gin from gout = dL/dRe N(x) + i dL/dIm N(x)."""
    ws = _nn_ws(op, True)
    _check(load().nn_backward(op.handle, _ptr(weights), _ptr(x), _ptr(gout), _ptr(dW),
                              _ptr(gin), 1 if f32_mixing else 0, _ptr(ws), ws.numel(),
                              _stream()), "nn_backward")


LOSS = {"error": 0, "dnorm": 1}


def nn_train_step(op: Op, weights, adam, step: int, lr: float, rhos, errs,
                  prec: str = "f64", loss: str = "dnorm") -> float:
    """One Adam step on a batch of (residual, error) fields of precision `prec`; returns
    the batch loss before the update. loss: "error" (|N(r) - e|^2/|e|^2) or "dnorm"
    (|D(N(r) - e)|^2/|De|^2)."""
    n = len(rhos)
    ws = _nn_ws(op, True, extra=8 * nn_weight_count() + 512)
    rp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in rhos])
    ep = (ctypes.c_void_p * n)(*[t.data_ptr() for t in errs])
    out = ctypes.c_double()
    _check(load().nn_train_step(op.handle, _ptr(weights), _ptr(adam), step, lr, rp, ep, n,
                                PREC[prec], LOSS[loss], ctypes.byref(out), _ptr(ws),
                                ws.numel(), _stream()), "nn_train_step")
    return out.value
