"""Thin ctypes binding of libppa.so (C ABI in include/ppa.h).

Argument marshalling only: every step of the method runs in the library (HIP
kernels on the device, small projected problems on the host in C++).  PyTorch
supplies device memory and the current stream.  There is no fallback: if the
built library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np
import torch  # loads torch's HIP runtime first, so libppa binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libppa.so")

PPA_OK = 0
PPA_WARN_DEGREE_REDUCED = 1
PPA_WARN_NOT_CONVERGED = 2
PPA_WARN_BREAKDOWN = 3
PPA_ERR_INVALID, PPA_ERR_HIP, PPA_ERR_WORKSPACE, PPA_ERR_NONFINITE = -1, -2, -3, -4
PPA_F64, PPA_F32, PPA_MIXED = 0, 1, 2
PPA_MATRIX_F32, PPA_MATRIX_WINDOW_FORCE, PPA_MATRIX_WINDOW_OFF, PPA_MATRIX_RING_FORCE = 1, 2, 4, 8
PPA_MATRIX_NO_TUNE = 16
PPA_MATRIX_RUNS_FORCE = 32
PPA_MATRIX_TWO_STEP = 64
_PREC = {"f64": PPA_F64, "f32": PPA_F32, "mixed": PPA_MIXED}

vp = C.c_void_p


class EigsOpts(C.Structure):
    _fields_ = [("m", C.c_int), ("k", C.c_int), ("nev", C.c_int), ("max_cycles", C.c_int),
                ("rtol", C.c_double), ("anorm", C.c_double), ("precision", C.c_int),
                ("flags", C.c_int)]


class EigsResult(C.Structure):
    _fields_ = [("lam_re", C.POINTER(C.c_double)), ("lam_im", C.POINTER(C.c_double)),
                ("resid", C.POINTER(C.c_double)), ("ritz_re", C.POINTER(C.c_double)),
                ("ritz_im", C.POINTER(C.c_double)), ("X_d", vp),
                ("nconv", C.c_int), ("cycles", C.c_int), ("mvps", C.c_int64),
                ("dots", C.c_int64), ("vops", C.c_int64), ("max_resid", C.c_double),
                ("fp32_cycles", C.c_int), ("reserved", C.c_int),
                ("spmv_passes", C.c_int64), ("spmv_passes_f32", C.c_int64), ("spmv_bytes", C.c_double),
                ("t_apply_ms", C.c_double), ("t_cgs_ms", C.c_double)]


class PolyBuildOpts(C.Structure):
    _fields_ = [("d", C.c_int), ("damp", C.c_int), ("alpha", C.c_double), ("test_m", C.c_int),
                ("test_k", C.c_int), ("test_nev", C.c_int), ("shift", C.c_double), ("flags", C.c_int)]


class PolyBuildInfo(C.Structure):
    _fields_ = [("degree", C.c_int), ("damp", C.c_int), ("attempts", C.c_int), ("held", C.c_int)]


class BatchRequest(C.Structure):
    _fields_ = [("n", C.c_int64), ("rowptr_d", vp), ("colind_d", vp), ("val_d", vp),
                ("anorm", C.c_double), ("d", C.c_int), ("m", C.c_int), ("k", C.c_int),
                ("nev", C.c_int), ("max_cycles", C.c_int), ("rtol", C.c_double),
                ("b_d", vp), ("v0_d", vp), ("ws_d", vp), ("ws_bytes", C.c_size_t)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run python -m paper_1806_08020_amd.build")
    lib = C.CDLL(LIB_PATH)
    i, i64, d, sz = C.c_int, C.c_int64, C.c_double, C.c_size_t
    P = C.POINTER
    sig = {
        "ppa_abi_version": (i, []),
        "ppa_last_error": (C.c_char_p, []),
        "ppa_matrix_create": (i, [i64, vp, vp, vp, vp, i, vp, P(vp)]),
        "ppa_matrix_destroy": (i, [vp]),
        "ppa_matrix_info": (i, [vp, P(i64), P(i64), P(d), P(i64)]),
        "ppa_matrix_spmv_variant": (i, [vp, i, P(i)]),
        "ppa_matrix_cache_policy": (i, [vp, i, P(i)]),
        "ppa_matrix_set_cache_policy": (i, [vp, i, i]),
        "ppa_matrix_spmv_blocks": (i, [vp, i, P(i)]),
        "ppa_matrix_set_spmv_blocks": (i, [vp, i, i]),
        "ppa_matrix_spmv_runs": (i, [vp, i, P(i), P(i64)]),
        "ppa_matrix_set_spmv_runs": (i, [vp, i, i]),
        "ppa_matrix_two_step": (i, [vp, i, P(i), P(i)]),
        "ppa_matrix_set_two_step": (i, [vp, i, i]),
        "ppa_poly_from_roots": (i, [i, P(d), P(d), i, P(d), P(d), P(vp)]),
        "ppa_poly_destroy": (i, [vp]),
        "ppa_poly_degree": (i, [vp, P(i), P(i)]),
        "ppa_poly_roots": (i, [vp, i, P(d), P(d), i, P(i)]),
        "ppa_poly_shift": (i, [vp, P(d)]),
        "ppa_poly_set_shift": (i, [vp, d]),
        "ppa_poly_build_ex_workspace_bytes": (i, [vp, P(PolyBuildOpts), i, P(sz)]),
        "ppa_poly_build_ex": (i, [vp, P(PolyBuildOpts), vp, vp, vp, sz, vp, P(vp), P(PolyBuildInfo)]),
        "ppa_poly_log10_pof": (i, [vp, i, P(d), i, P(i)]),
        "ppa_poly_stabilize": (i, [vp, i, P(vp), P(i)]),
        "ppa_poly_build_workspace_bytes": (i, [vp, i, i, P(sz)]),
        "ppa_poly_build": (i, [vp, i, vp, vp, sz, vp, P(vp)]),
        "ppa_poly_build_double": (i, [vp, i, i, vp, vp, sz, vp, P(vp)]),
        "ppa_poly_apply_workspace_bytes": (i, [vp, vp, i, P(sz)]),
        "ppa_poly_apply": (i, [vp, vp, i, vp, vp, vp, sz, vp]),
        "ppa_poly_apply_bytes": (i, [vp, vp, i, P(d)]),
        "ppa_poly_apply_noalloc": (i, [vp, vp, i, vp, vp, vp]),
        "ppa_fused_spmv": (i, [vp, i, i, d, vp, d, vp, d, vp, d, vp, vp, vp]),
        "ppa_cgs2_workspace_bytes": (i, [i64, i, P(sz)]),
        "ppa_cgs2": (i, [i64, i, vp, i64, vp, P(d), P(d), vp, sz, vp]),
        "ppa_gemm_workspace_bytes": (i, [i, i, P(sz)]),
        "ppa_gemm_tall": (i, [i64, i, i, vp, i64, P(d), vp, i64, vp, sz, vp]),
        "ppa_eigs_workspace_bytes": (i, [vp, vp, P(EigsOpts), P(sz)]),
        "ppa_eigs": (i, [vp, vp, P(EigsOpts), vp, vp, sz, vp, P(EigsResult)]),
        "ppa_batch_workspace_bytes": (i, [i64, i, i, i, P(sz)]),
        "ppa_batch_workspace_bytes_ex": (i, [i64, i64, i, i, i, i, P(sz)]),
        "ppa_batch_create": (i, [i, vp, P(vp)]),
        "ppa_batch_destroy": (i, [vp]),
        "ppa_batch_submit": (i, [vp, P(BatchRequest), P(i)]),
        "ppa_batch_submit_ex": (i, [vp, P(BatchRequest), i, P(i)]),
        "ppa_batch_step": (i, [vp, P(i), i, P(i), P(i)]),
        "ppa_batch_result": (i, [vp, i, P(EigsResult)]),
        "ppa_dense_eig": (i, [i, P(d), P(d), P(d), P(d), P(d)]),
        "ppa_leja_order": (i, [i, P(d), P(d)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


class PPAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libppa status {status}: {msg}")
        self.status = status


def _check(st):
    if st < 0:
        raise PPAError(st, _lib.ppa_last_error().decode())
    return st


def _stream():
    return vp(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return vp(t.data_ptr()) if t is not None else None


def _dptr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _workspace(nbytes):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


def abi_version() -> int:
    return _lib.ppa_abi_version()


# ---------------------------------------------------------------- matrix
class Matrix:
    """Device CSR matrix handle.  ``csr`` is a workloads.CSR (host arrays);
    the device copies are owned by this object and borrowed by the handle."""

    def __init__(self, csr, want_f32: bool = False, window: str = "auto", tune: bool = True,
                 two_step: bool = False):
        """window: "auto" (time the SpMV variants on large matrices),
        "force" (LDS-windowed whenever it fits), "ring" (sliding window
        whenever it fits), "runs" (plain kernel with column runs staged in
        LDS) or "off" (plain kernel only, global gathers).  tune=False skips the
        timing at creation (size-rule cache policy, large blocks).  two_step:
        build (and use) two factors of pi per pass where the bandwidth
        allows it (ppa_matrix_two_step)."""
        dev = torch.device("cuda")
        self.n = int(csr.n)
        self.rowptr = torch.as_tensor(np.asarray(csr.rowptr, dtype=np.int32)).to(dev)
        self.colind = torch.as_tensor(np.asarray(csr.colind, dtype=np.int32)).to(dev)
        self.vals = torch.as_tensor(np.asarray(csr.vals, dtype=np.float64)).to(dev)
        if self.colind.numel() == 0:      # keep valid pointers for empty matrices
            self.colind = torch.zeros(1, dtype=torch.int32, device=dev)
            self.vals = torch.zeros(1, dtype=torch.float64, device=dev)
        self.vals32 = self.vals.float() if want_f32 else None
        h = vp()
        flags = {"auto": 0, "force": PPA_MATRIX_WINDOW_FORCE, "ring": PPA_MATRIX_RING_FORCE,
                 "off": PPA_MATRIX_WINDOW_OFF, "runs": PPA_MATRIX_RUNS_FORCE}[window]
        if not tune:
            flags |= PPA_MATRIX_NO_TUNE
        if two_step:
            flags |= PPA_MATRIX_TWO_STEP
        _check(_lib.ppa_matrix_create(self.n, _ptr(self.rowptr), _ptr(self.colind), _ptr(self.vals),
                                      _ptr(self.vals32), flags, _stream(), C.byref(h)))
        self.h = h
        n, nnz, nrm, nb = C.c_int64(), C.c_int64(), C.c_double(), C.c_int64()
        _check(_lib.ppa_matrix_info(self.h, C.byref(n), C.byref(nnz), C.byref(nrm), C.byref(nb)))
        self.nnz, self.norm_inf, self.nblocks = nnz.value, nrm.value, nb.value

    @property
    def has_f32(self):
        return self.vals32 is not None

    def windowed(self, precision: str = "f64") -> bool:
        """True when either LDS-staged SpMV variant is in use."""
        return self.spmv_variant(precision) != "plain"

    SPMV_VARIANTS = ("plain", "window", "ring")

    def spmv_variant(self, precision: str = "f64") -> str:
        """SpMV kernel in use: "plain", "window" (per-block LDS window) or
        "ring" (sliding window)."""
        w = C.c_int()
        _check(_lib.ppa_matrix_spmv_variant(self.h, _PREC[precision], C.byref(w)))
        return self.SPMV_VARIANTS[w.value]

    CACHE_POLICIES = ("stream", "keep", "keep_ntst")

    def cache_policy(self, precision: str = "f64") -> str:
        """Cache policy of the plain SpMV kernel: "stream", "keep" or "keep_ntst"."""
        c = C.c_int()
        _check(_lib.ppa_matrix_cache_policy(self.h, _PREC[precision], C.byref(c)))
        return self.CACHE_POLICIES[c.value]

    def set_cache_policy(self, policy: str, precision: str = "f64") -> None:
        _check(_lib.ppa_matrix_set_cache_policy(self.h, _PREC[precision],
                                                self.CACHE_POLICIES.index(policy)))

    def spmv_blocks(self, precision: str = "f64") -> int:
        """Nonzeros per block of the plain SpMV kernel (2048 or 256)."""
        c = C.c_int()
        _check(_lib.ppa_matrix_spmv_blocks(self.h, _PREC[precision], C.byref(c)))
        return c.value

    def set_spmv_blocks(self, nnz_per_block: int, precision: str = "f64") -> None:
        _check(_lib.ppa_matrix_set_spmv_blocks(self.h, _PREC[precision], int(nnz_per_block)))

    def spmv_runs(self, precision: str = "f64"):
        """(on, blocks with runs): whether the plain kernel stages column
        runs in LDS, and how many large blocks have runs within budget."""
        on, nb = C.c_int(), C.c_int64()
        _check(_lib.ppa_matrix_spmv_runs(self.h, _PREC[precision], C.byref(on), C.byref(nb)))
        return bool(on.value), nb.value

    def set_spmv_runs(self, on: bool, precision: str = "f64") -> None:
        _check(_lib.ppa_matrix_set_spmv_runs(self.h, _PREC[precision], int(bool(on))))

    def two_step(self, precision: str = "f64"):
        """(on, bandwidth): whether pi is applied two factors per pass, and
        the bandwidth found at creation (-1 when no records were built)."""
        on, bw = C.c_int(), C.c_int()
        _check(_lib.ppa_matrix_two_step(self.h, _PREC[precision], C.byref(on), C.byref(bw)))
        return bool(on.value), bw.value

    def set_two_step(self, on: bool, precision: str = "f64") -> None:
        _check(_lib.ppa_matrix_set_two_step(self.h, _PREC[precision], int(bool(on))))

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:   # the module may already be torn down at exit
            _lib.ppa_matrix_destroy(h)
            self.h = None


# ---------------------------------------------------------------- polynomial
class Poly:
    def __init__(self, h, status=PPA_OK):
        self.h = h
        self.status = status
        deg, d1 = C.c_int(), C.c_int()
        _check(_lib.ppa_poly_degree(h, C.byref(deg), C.byref(d1)))
        self.degree, self.d1 = deg.value, d1.value

    @classmethod
    def from_roots(cls, roots, roots1=None):
        r = np.asarray(roots, dtype=complex)
        re, pre = _dptr(r.real)
        im, pim = _dptr(r.imag)
        if roots1 is not None:
            r1 = np.asarray(roots1, dtype=complex)
            re1, pre1 = _dptr(r1.real)
            im1, pim1 = _dptr(r1.imag)
            d1 = r1.size
        else:
            pre1 = pim1 = None
            d1 = 0
        h = vp()
        _check(_lib.ppa_poly_from_roots(r.size, pre, pim, d1, pre1, pim1, C.byref(h)))
        return cls(h)

    @classmethod
    def build(cls, A: Matrix, d: int, b: torch.Tensor, lowsync: bool = False):
        """GMRES(d) polynomial from b (``lowsync``: the GMRES cycle uses the
        delayed-reorthogonalisation Gram-Schmidt)."""
        if lowsync:
            return cls.build_ex(A, d, b, lowsync=True)[0]
        nb = C.c_size_t()
        _check(_lib.ppa_poly_build_workspace_bytes(A.h, d, 0, C.byref(nb)))
        ws = _workspace(nb.value)
        h = vp()
        st = _check(_lib.ppa_poly_build(A.h, d, _ptr(b), _ptr(ws), ws.numel(), _stream(), C.byref(h)))
        return cls(h, st)

    @classmethod
    def build_double(cls, A: Matrix, d1: int, d2: int, b: torch.Tensor):
        nb = C.c_size_t()
        _check(_lib.ppa_poly_build_workspace_bytes(A.h, max(d1, d2), 1, C.byref(nb)))
        ws = _workspace(nb.value)
        h = vp()
        st = _check(_lib.ppa_poly_build_double(A.h, d1, d2, _ptr(b), _ptr(ws), ws.numel(), _stream(),
                                               C.byref(h)))
        return cls(h, st)

    @classmethod
    def build_ex(cls, A: Matrix, d: int, b: torch.Tensor, b2: torch.Tensor | None = None,
                 damp: int = 0, alpha: float = 0.0, test=None, shift: float = 0.0,
                 lowsync: bool = False):
        """GMRES polynomial with the safeguards of sections 5-6: damped start
        vector A^damp b (+ alpha b), optional second start vector b2, optional
        Ideal-Order-Condition test ``test = (m, k, nev)``, target ``shift``
        (the polynomial acts on A - shift I).  Returns (Poly, info)."""
        tm, tk, tn = test if test is not None else (0, 0, 0)
        o = PolyBuildOpts(d, damp, alpha, tm, tk, tn, shift, 4 if lowsync else 0)
        nb = C.c_size_t()
        _check(_lib.ppa_poly_build_ex_workspace_bytes(A.h, C.byref(o), int(b2 is not None), C.byref(nb)))
        ws = _workspace(nb.value)
        h = vp()
        info = PolyBuildInfo()
        st = _check(_lib.ppa_poly_build_ex(A.h, C.byref(o), _ptr(b), _ptr(b2), _ptr(ws), ws.numel(),
                                           _stream(), C.byref(h), C.byref(info)))
        return cls(h, st), dict(degree=info.degree, damp=info.damp, attempts=info.attempts,
                                held=info.held)

    @property
    def shift(self) -> float:
        x = C.c_double()
        _check(_lib.ppa_poly_shift(self.h, C.byref(x)))
        return x.value

    @shift.setter
    def shift(self, mu: float):
        _check(_lib.ppa_poly_set_shift(self.h, float(mu)))

    def log10_pof(self, level: int = 2) -> np.ndarray:
        """log10 pof(j) of the roots of ``level`` in application order."""
        cnt = self.degree if level == 2 else self.d1
        out = np.zeros(max(cnt, 1))
        c = C.c_int()
        _check(_lib.ppa_poly_log10_pof(self.h, level, out.ctypes.data_as(C.POINTER(C.c_double)),
                                       out.size, C.byref(c)))
        return out[: c.value]

    def stabilized(self, level: int = 2):
        """(new Poly with the section-7 extra roots at ``level``, roots added)."""
        h = vp()
        added = C.c_int()
        _check(_lib.ppa_poly_stabilize(self.h, level, C.byref(h), C.byref(added)))
        return Poly(h), added.value

    def roots(self, level: int = 2) -> np.ndarray:
        cnt = self.degree if level == 2 else self.d1
        re = np.zeros(max(cnt, 1))
        im = np.zeros(max(cnt, 1))
        c = C.c_int()
        _check(_lib.ppa_poly_roots(self.h, level, re.ctypes.data_as(C.POINTER(C.c_double)),
                                   im.ctypes.data_as(C.POINTER(C.c_double)), re.size, C.byref(c)))
        return (re + 1j * im)[: c.value]

    @property
    def is_double(self):
        return self.d1 > 0

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.ppa_poly_destroy(h)
            self.h = None


def apply(A: Matrix, p: Poly, v: torch.Tensor, precision: str = "f64", out=None, ws=None):
    """y = pi(A) v on the device (FP64 or FP32 vectors)."""
    prec = _PREC[precision]
    dt = torch.float64 if prec == PPA_F64 else torch.float32
    if v.dtype != dt or not v.is_cuda or v.numel() != A.n:
        raise ValueError("v must be a contiguous device vector of length n and matching dtype")
    y = torch.empty_like(v) if out is None else out
    if ws is None:
        ws = apply_workspace(A, p, precision)
    _check(_lib.ppa_poly_apply(A.h, p.h, prec, _ptr(v), _ptr(y), _ptr(ws), ws.numel(), _stream()))
    return y


NOALLOC_SCRATCH_BYTES = 64 << 20


def apply_noalloc(A: Matrix, p: Poly, v: torch.Tensor, precision: str = "f64", out=None):
    """y = pi(A) v through ppa_poly_apply_noalloc: the chain's temporaries live
    in the library's static per-device scratch array (no workspace)."""
    prec = _PREC[precision]
    dt = torch.float64 if prec == PPA_F64 else torch.float32
    if v.dtype != dt or not v.is_cuda or v.numel() != A.n:
        raise ValueError("v must be a contiguous device vector of length n and matching dtype")
    y = torch.empty_like(v) if out is None else out
    _check(_lib.ppa_poly_apply_noalloc(A.h, p.h, prec, _ptr(v), _ptr(y), _stream()))
    return y


def apply_bytes(A: Matrix, p: Poly, precision: str = "f64") -> float:
    """Algorithmic HBM bytes of one pi(A)v application (nothing is launched)."""
    b = C.c_double()
    _check(_lib.ppa_poly_apply_bytes(A.h, p.h, _PREC[precision], C.byref(b)))
    return b.value


def apply_workspace(A: Matrix, p: Poly, precision: str = "f64"):
    nb = C.c_size_t()
    _check(_lib.ppa_poly_apply_workspace_bytes(A.h, p.h, _PREC[precision], C.byref(nb)))
    return _workspace(nb.value)


def fused_spmv(A: Matrix, alpha, x, beta, u, gamma=0.0, z=None, delta=0.0, z2=None, out=None,
               out_dtype=None):
    """out = alpha x + beta (A u) + gamma z + delta z2 (one fused pass)."""
    in_f32 = u.dtype == torch.float32
    odt = out_dtype or u.dtype
    o = torch.empty(A.n, dtype=odt, device=u.device) if out is None else out
    _check(_lib.ppa_fused_spmv(A.h, int(in_f32), int(o.dtype == torch.float32), alpha, _ptr(x), beta,
                               _ptr(u), gamma, _ptr(z), delta, _ptr(z2), _ptr(o), _stream()))
    return o


def cgs2(V: torch.Tensor, j: int, w: torch.Tensor):
    """Orthogonalise w (in place) against the first j columns of V, given as
    a (ncols, ld) device tensor (row c = column c).  Returns (h[0..j], ||w_in||)."""
    n = w.numel()
    ld = V.shape[1]
    nb = C.c_size_t()
    _check(_lib.ppa_cgs2_workspace_bytes(n, j, C.byref(nb)))
    ws = _workspace(nb.value)
    h = np.zeros(j + 1)
    w0 = C.c_double()
    _check(_lib.ppa_cgs2(n, j, _ptr(V), ld, _ptr(w), h.ctypes.data_as(C.POINTER(C.c_double)),
                         C.byref(w0), _ptr(ws), ws.numel(), _stream()))
    return h, w0.value


def gemm_tall(V: torch.Tensor, Q: np.ndarray, n: int) -> torch.Tensor:
    """C = V[:, :kin] Q with V given as (kin, ld) device tensor (row c = column c
    of the column-major block); returns C as (kout, n)."""
    Q = np.asfortranarray(Q, dtype=np.float64)
    kin, kout = Q.shape
    ld = V.shape[1]
    C_ = torch.empty((kout, n), dtype=torch.float64, device="cuda")
    nb = C.c_size_t()
    _check(_lib.ppa_gemm_workspace_bytes(kin, kout, C.byref(nb)))
    ws = _workspace(nb.value)
    qf = np.ascontiguousarray(Q.T).ravel()   # column-major kin x kout
    _check(_lib.ppa_gemm_tall(n, kin, kout, _ptr(V), ld, qf.ctypes.data_as(C.POINTER(C.c_double)),
                              _ptr(C_), n, _ptr(ws), ws.numel(), _stream()))
    torch.cuda.current_stream().synchronize()
    return C_


@dataclass
class EigsOut:
    status: int
    mu: np.ndarray
    resid: np.ndarray
    nu: np.ndarray
    nconv: int
    cycles: int
    mvps: int
    dots: int
    vops: int
    max_resid: float
    fp32_cycles: int
    spmv_passes: int = 0
    spmv_passes_f32: int = 0
    spmv_bytes: float = 0.0
    t_apply_ms: float = 0.0
    t_cgs_ms: float = 0.0
    X: torch.Tensor | None = None
    converged: bool = field(default=False)


def eigs_workspace(A: Matrix, p: Poly | None, m, k, nev, precision="f64"):
    o = EigsOpts(m, k, nev, 1, 1e-8, 0.0, _PREC[precision], 0)
    nb = C.c_size_t()
    _check(_lib.ppa_eigs_workspace_bytes(A.h, p.h if p else None, C.byref(o), C.byref(nb)))
    return _workspace(nb.value)


def eigs(A: Matrix, p: Poly | None, v0: torch.Tensor, m: int, k: int, nev: int, rtol: float = 1e-8,
         max_cycles: int = 100, precision: str = "f64", anorm: float = 0.0,
         want_vectors: bool = False, ws=None, timing: bool = False,
         harmonic: bool = False, lowsync: bool = False, graph: bool = False) -> EigsOut:
    """Thick-restarted Arnoldi(m,k) on pi(A) for nev eigenpairs of A
    (``harmonic``: restart with harmonic Ritz vectors; ``lowsync``: Gram-Schmidt
    with the reorthogonalisation delayed by one step; ``graph``: replay each
    cycle's Krylov steps from a HIP graph)."""
    o = EigsOpts(m, k, nev, max_cycles, rtol, anorm, _PREC[precision],
                 (1 if timing else 0) | (2 if harmonic else 0) | (4 if lowsync else 0)
                 | (8 if graph else 0))
    if ws is None:
        nb = C.c_size_t()
        _check(_lib.ppa_eigs_workspace_bytes(A.h, p.h if p else None, C.byref(o), C.byref(nb)))
        ws = _workspace(nb.value)
    lre, lim, res, nre, nim = (np.zeros(nev) for _ in range(5))
    X = torch.empty((nev, A.n), dtype=torch.complex128, device="cuda") if want_vectors else None
    r = EigsResult()
    P = C.POINTER(C.c_double)
    r.lam_re, r.lam_im, r.resid = lre.ctypes.data_as(P), lim.ctypes.data_as(P), res.ctypes.data_as(P)
    r.ritz_re, r.ritz_im = nre.ctypes.data_as(P), nim.ctypes.data_as(P)
    r.X_d = X.data_ptr() if X is not None else None
    st = _check(_lib.ppa_eigs(A.h, p.h if p else None, C.byref(o), _ptr(v0), _ptr(ws), ws.numel(),
                              _stream(), C.byref(r)))
    return EigsOut(status=st, mu=lre + 1j * lim, resid=res.copy(), nu=nre + 1j * nim, nconv=r.nconv,
                   cycles=r.cycles, mvps=r.mvps, dots=r.dots, vops=r.vops, max_resid=r.max_resid,
                   fp32_cycles=r.fp32_cycles, spmv_passes=r.spmv_passes,
                   spmv_passes_f32=r.spmv_passes_f32, spmv_bytes=r.spmv_bytes, t_apply_ms=r.t_apply_ms,
                   t_cgs_ms=r.t_cgs_ms, X=X, converged=(st == PPA_OK))


# ---------------------------------------------------------------- batched engine
PPA_ERR_BUSY = -7


def batch_workspace_bytes(n: int, d: int, m: int, nev: int, nnz: int = 0, precision: str = "f64") -> int:
    """Workspace of one batched request; "mixed" also holds FP32 values (nnz)
    and the FP32 chain vectors."""
    nb = C.c_size_t()
    if precision == "f64":
        _check(_lib.ppa_batch_workspace_bytes(n, d, m, nev, C.byref(nb)))
    else:
        _check(_lib.ppa_batch_workspace_bytes_ex(n, nnz, d, m, nev, _PREC[precision], C.byref(nb)))
    return nb.value


class Batch:
    """Batched engine for many small solves: one launch per step advances
    every admitted solve by one phase (one workgroup each).  All work goes to
    the stream current at construction (or the given torch stream)."""

    def __init__(self, max_slots: int, stream=None):
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = vp()
        _check(_lib.ppa_batch_create(max_slots, vp(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.max_slots = max_slots
        self._keep = {}
        self._fin = (C.c_int * max_slots)()

    def submit(self, rowptr, colind, vals, d, m, k, nev, b, v0, rtol=1e-8, max_cycles=50,
               anorm=0.0, ws=None, precision="f64"):
        """Admit one solve; device tensors stay referenced until its result is
        taken.  precision: "f64" or "mixed" (FP32 pi(A)v, closing FP64
        Rayleigh-Ritz).  Returns the slot, or None when the engine is full."""
        n = rowptr.numel() - 1
        if precision not in ("f64", "mixed"):
            raise ValueError("precision must be 'f64' or 'mixed'")
        if ws is None:
            ws = _workspace(batch_workspace_bytes(n, d, m, nev, vals.numel(), precision))
        rq = BatchRequest(n, _ptr(rowptr), _ptr(colind), _ptr(vals), anorm, d, m, k, nev, max_cycles,
                          rtol, _ptr(b), _ptr(v0), _ptr(ws), ws.numel())
        slot = C.c_int(-1)
        if precision == "f64":
            st = _lib.ppa_batch_submit(self.h, C.byref(rq), C.byref(slot))
        else:
            st = _lib.ppa_batch_submit_ex(self.h, C.byref(rq), _PREC[precision], C.byref(slot))
        if st == PPA_ERR_BUSY:
            return None
        _check(st)
        self._keep[slot.value] = (rowptr, colind, vals, b, v0, ws, nev)
        return slot.value

    def step(self):
        """One batched launch; returns (finished slots, number of active solves)."""
        nf, na = C.c_int(), C.c_int()
        _check(_lib.ppa_batch_step(self.h, self._fin, self.max_slots, C.byref(nf), C.byref(na)))
        return [self._fin[i] for i in range(min(nf.value, self.max_slots))], na.value

    def result(self, slot: int) -> EigsOut:
        nev = self._keep[slot][6]
        lre, lim, res, nre, nim = (np.zeros(nev) for _ in range(5))
        r = EigsResult()
        P = C.POINTER(C.c_double)
        r.lam_re, r.lam_im, r.resid = lre.ctypes.data_as(P), lim.ctypes.data_as(P), res.ctypes.data_as(P)
        r.ritz_re, r.ritz_im = nre.ctypes.data_as(P), nim.ctypes.data_as(P)
        r.X_d = None
        st = _check(_lib.ppa_batch_result(self.h, slot, C.byref(r)))
        del self._keep[slot]
        return EigsOut(status=st, mu=lre + 1j * lim, resid=res.copy(), nu=nre + 1j * nim, nconv=r.nconv,
                       cycles=r.cycles, mvps=r.mvps, dots=r.dots, vops=r.vops, max_resid=r.max_resid,
                       fp32_cycles=r.fp32_cycles, spmv_passes=r.spmv_passes,
                       spmv_passes_f32=r.spmv_passes_f32, converged=(st == PPA_OK))

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.ppa_batch_destroy(h)
            self.h = None


# ---------------------------------------------------------------- host helpers
def dense_eig(a: np.ndarray, vectors: bool = True):
    a = np.asfortranarray(a, dtype=np.float64)
    n = a.shape[0]
    wr, wi = np.zeros(n), np.zeros(n)
    vr = np.zeros((n, n), order="F") if vectors else None
    vi = np.zeros((n, n), order="F") if vectors else None
    P = C.POINTER(C.c_double)
    _check(_lib.ppa_dense_eig(n, a.ctypes.data_as(P), wr.ctypes.data_as(P), wi.ctypes.data_as(P),
                              vr.ctypes.data_as(P) if vectors else None,
                              vi.ctypes.data_as(P) if vectors else None))
    w = wr + 1j * wi
    return (w, vr + 1j * vi) if vectors else w


def leja_order(roots) -> np.ndarray:
    r = np.asarray(roots, dtype=complex)
    re = np.ascontiguousarray(r.real.copy())
    im = np.ascontiguousarray(r.imag.copy())
    P = C.POINTER(C.c_double)
    _check(_lib.ppa_leja_order(r.size, re.ctypes.data_as(P), im.ctypes.data_as(P)))
    return re + 1j * im
