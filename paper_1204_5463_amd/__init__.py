"""Python binding of libdwsap, the MI355X SAP-preconditioned FGMRES-DR solver
for the Wilson-Dirac operator (arXiv:1204.5463).

This module only marshals arguments: it loads the HIP library, passes
device pointers of PyTorch tensors and the current HIP stream, and turns
status codes into exceptions. Every step of the method runs in the
library's kernels. PyTorch supplies device memory (through its caching
allocator, handed to the library as an allocator callback) and streams.

Field layout at this boundary: complex128 tensors on the GPU,
  spinor  psi[(rhs,) t, z, y, x, spin, colour]
  gauge   U[mu, t, z, y, x, a, b]          (mu = x, y, z, t)
with lattice extents L = (Lx, Ly, Lz, Lt).
"""
from __future__ import annotations

import atexit
import ctypes
import dataclasses
import os
import weakref

import torch

__all__ = [
    "DW_PREC_F64", "DW_PREC_F32", "DW_PREC_F16", "DW_PREC_BF16", "PREC_NAMES",
    "DwError", "NotConverged", "Context", "Field", "SapParams", "SolverParams", "SolveStats", "Server",
    "TuneSpace", "TuneCache", "autotune",
    "lib", "load",
]

DW_OK, DW_EINVAL, DW_ENOMEM, DW_EHIP, DW_ENOTCONV, DW_EBUSY, DW_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
DW_PREC_F64, DW_PREC_F32, DW_PREC_F16, DW_PREC_BF16 = 0, 1, 2, 3
SOLVE_GRAPHS, SOLVE_V32, SOLVE_INJECT, SOLVE_A32 = 1, 2, 4, 8
PREC_NAMES = {"f64": DW_PREC_F64, "f32": DW_PREC_F32, "f16": DW_PREC_F16, "bf16": DW_PREC_BF16}
PAIR_BYTES = {DW_PREC_F64: 16, DW_PREC_F32: 8, DW_PREC_F16: 4, DW_PREC_BF16: 4}

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdwsap.so")


class DwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dwsap status {status}: {msg}")
        self.status = status


class NotConverged(DwError):
    pass


class _SapParams(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32 * 4), ("ncycles", ctypes.c_int32), ("nmr", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("reserved", ctypes.c_int32), ("mr_reduction", ctypes.c_double)]


class _SolverParams(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("k", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("shared_defl", ctypes.c_int32), ("tol", ctypes.c_double), ("restart_t", ctypes.c_double),
                ("sap", _SapParams), ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


KCLASS = {"dslash_f64": 0, "dslash_lowp": 1, "sap": 2, "dots": 3, "reduce": 4, "subcols": 5, "scale": 6,
          "combine": 7, "rotate": 8, "convert": 9, "dense": 10}


class _KStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int32), ("iterations", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("clean_restarts", ctypes.c_int32), ("true_relres", ctypes.c_double),
                ("implicit_relres", ctypes.c_double), ("seconds", ctypes.c_double)]


class _ServerParams(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("queue_capacity", ctypes.c_int32), ("budget_bytes", ctypes.c_double)]


class _Request(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("block", ctypes.c_int32 * 4), ("m0", ctypes.c_double),
                ("csw", ctypes.c_double), ("U", ctypes.c_void_p), ("nrhs", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("b", ctypes.c_void_p), ("x", ctypes.c_void_p), ("params", _SolverParams)]


class _ReqTimes(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_double), ("running", ctypes.c_double), ("latency", ctypes.c_double)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


class _TuneSpace(ctypes.Structure):
    _fields_ = [("nblocks", ctypes.c_int32), ("blocks", (ctypes.c_int32 * 4) * 16),
                ("nmr_min", ctypes.c_int32), ("nmr_max", ctypes.c_int32),
                ("s_min", ctypes.c_int32), ("s_max", ctypes.c_int32),
                ("nmk", ctypes.c_int32), ("mk", (ctypes.c_int32 * 2) * 8),
                ("repeats", ctypes.c_int32), ("passes", ctypes.c_int32), ("iter_cap", ctypes.c_double)]


class _TuneTrial(ctypes.Structure):
    _fields_ = [("params", _SolverParams), ("converged", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("seconds", ctypes.c_double)]

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("release", _FREE_FN), ("user", ctypes.c_void_p)]


@dataclasses.dataclass
class SapParams:
    """SAP preconditioner (Alg. 2): block extents, cycles s, MR steps, storage precision.

    mr_reduction > 0 makes the block solves inexact in the adaptive sense of
    Section 3: each block stops at the first MR step whose residual is at most
    mr_reduction times its right-hand side's norm (nmr bounds the steps)."""
    block: tuple = (4, 4, 4, 4)
    ncycles: int = 1
    nmr: int = 4
    storage: int = DW_PREC_F64
    mr_reduction: float = 0.0

    def _c(self):
        p = _SapParams()
        for i in range(4):
            p.block[i] = int(self.block[i])
        p.ncycles, p.nmr, p.storage, p.reserved = int(self.ncycles), int(self.nmr), int(self.storage), 0
        p.mr_reduction = float(self.mr_reduction)
        return p


@dataclasses.dataclass
class SolverParams:
    """FGMRES-DR(m, k) (Alg. 4) with the Section 4.7 clean-restart threshold."""
    m: int = 20
    k: int = 5
    max_iter: int = 10000
    tol: float = 1e-10
    restart_t: float = 5.0
    sap: SapParams = dataclasses.field(default_factory=SapParams)
    shared_defl: int = 0
    # SOLVE_GRAPHS: replay captured restart cycles, kept with the field (non-default stream); SOLVE_V32: FP32 basis;
    # SOLVE_INJECT: explicit residual also in G_{k+1} and v_{k+1} at deflated restarts (Section 4.7)
    flags: int = 0

    def _c(self):
        p = _SolverParams()
        p.m, p.k, p.max_iter, p.shared_defl = int(self.m), int(self.k), int(self.max_iter), int(self.shared_defl)
        p.tol, p.restart_t = float(self.tol), float(self.restart_t)
        p.sap = self.sap._c()
        p.flags, p.reserved = int(self.flags), 0
        return p


@dataclasses.dataclass
class SolveStats:
    converged: bool
    iterations: int
    cycles: int
    clean_restarts: int
    true_relres: float
    implicit_relres: float
    seconds: float


_lib = None

# Handles still open when the interpreter exits are closed before it tears
# down (the library frees device memory through PyTorch's allocator, which
# must still be alive then): servers first, then fields, then contexts.
_live = {"server": weakref.WeakSet(), "field": weakref.WeakSet(), "context": weakref.WeakSet()}


@atexit.register
def _close_all():
    for kind in ("server", "field", "context"):
        for obj in list(_live[kind]):
            try:
                obj.close()
            except Exception:
                pass


def load(path: str = LIB_PATH):
    """Load libdwsap.so. Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libdwsap.so not found at {path}; build it with `python -m paper_1204_5463_amd.build`")
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_int32
    sig = {
        "dw_last_error": (ctypes.c_char_p, []),
        "dw_ctx_create": (st, [i32, ctypes.POINTER(_Allocator), ctypes.POINTER(vp)]),
        "dw_ctx_destroy": (st, [vp]),
        "dw_field_create": (st, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), vp, vp, ctypes.POINTER(vp)]),
        "dw_field_destroy": (st, [vp]),
        "dw_field_set_clover": (st, [vp, dbl, vp]),
        "dw_field_volume": (i64, [vp]),
        "dw_apply": (st, [vp, dbl, vp, vp, i32, vp]),
        "dw_apply_ex": (st, [vp, dbl, i32, vp, vp, i32, vp]),
        "dw_apply_noalloc": (st, [vp, dbl, vp, vp, i32, vp]),
        "dw_apply_noalloc_max_bytes": (ctypes.c_size_t, []),
        "dw_dense_lsq": (st, [vp, i32, vp, vp, vp, ctypes.POINTER(dbl)]),
        "dw_dense_restart": (st, [vp, i32, i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(i32)]),
        "dw_internal_bytes": (ctypes.c_size_t, [vp, i32, i32]),
        "dw_pack": (st, [vp, i32, vp, vp, i32, vp]),
        "dw_unpack": (st, [vp, i32, vp, vp, i32, vp]),
        "sap_precondition": (st, [vp, dbl, ctypes.POINTER(_SapParams), vp, vp, i32, vp]),
        "sap_solve": (st, [vp, dbl, ctypes.POINTER(_SapParams), vp, vp, i32, ctypes.POINTER(dbl), vp]),
        "fgmresdr_solve": (st, [vp, dbl, ctypes.POINTER(_SolverParams), vp, vp, i32, ctypes.POINTER(_Stats), vp]),
        "dw_profile_enable": (st, [vp, i32]),
        "dw_profile_get": (st, [vp, i32, ctypes.POINTER(_KStats)]),
        "dw_profile_reset": (st, [vp]),
        "dw_server_create": (st, [vp, ctypes.POINTER(_ServerParams), ctypes.POINTER(vp)]),
        "dw_server_destroy": (st, [vp]),
        "dw_request_footprint": (ctypes.c_size_t, [ctypes.POINTER(_Request)]),
        "solve_submit": (st, [vp, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)]),
        "solve_poll": (st, [vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(_Stats),
                            ctypes.POINTER(_ReqTimes)]),
        "dw_autotune": (st, [vp, ctypes.POINTER(i32), vp, dbl, dbl, ctypes.POINTER(_SolverParams),
                             ctypes.POINTER(_TuneSpace), vp, vp, i32, ctypes.POINTER(_TuneTrial), i32,
                             ctypes.POINTER(i32), ctypes.POINTER(_SolverParams), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def lib():
    return load()


def _check(status, what=""):
    if status != DW_OK:
        msg = lib().dw_last_error().decode(errors="replace")
        if status == DW_ENOTCONV:
            raise NotConverged(status, msg)
        raise DwError(status, f"{what}: {msg}" if what else msg)


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev_ptr(t: torch.Tensor, dtype=torch.complex128):
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A library context on one device, allocating through PyTorch's caching allocator."""

    def __init__(self, device: int = 0, use_torch_allocator: bool = True):
        L = lib()
        self.device = device
        self._alloc = None
        if use_torch_allocator:
            dev = device

            def _a(nbytes, stream, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
                except Exception:
                    return None

            def _f(ptr, stream, user):
                torch.cuda.caching_allocator_delete(int(ptr))

            self._afn, self._ffn = _ALLOC_FN(_a), _FREE_FN(_f)
            self._alloc = _Allocator(self._afn, self._ffn, None)
        h = ctypes.c_void_p()
        _check(L.dw_ctx_create(device, ctypes.byref(self._alloc) if self._alloc else None, ctypes.byref(h)),
               "dw_ctx_create")
        self.handle = h
        _live["context"].add(self)

    def profile(self, on: bool = True):
        """Per-kernel-class HIP-event timing of every launch made for this context."""
        _check(lib().dw_profile_enable(self.handle, 1 if on else 0), "dw_profile_enable")

    def profile_reset(self):
        _check(lib().dw_profile_reset(self.handle), "dw_profile_reset")

    def profile_stats(self):
        """{class name: dict(launches, ms, bytes, flops)} accumulated since the last reset."""
        out = {}
        for name, kc in KCLASS.items():
            k = _KStats()
            _check(lib().dw_profile_get(self.handle, kc, ctypes.byref(k)), "dw_profile_get")
            out[name] = {"launches": int(k.launches), "ms": k.ms, "bytes": k.bytes, "flops": k.flops}
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().dw_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Field:
    """A gauge field tiled into SAP blocks (the library keeps its own copies)."""

    def __init__(self, ctx: Context, L, block, U: torch.Tensor, stream=None):
        self.ctx = ctx
        self.L = tuple(int(v) for v in L)
        self.block = tuple(int(v) for v in block)
        Lx, Ly, Lz, Lt = self.L
        if tuple(U.shape) != (4, Lt, Lz, Ly, Lx, 3, 3):
            raise ValueError(f"gauge shape {tuple(U.shape)} does not match L={self.L}")
        La = (ctypes.c_int32 * 4)(*self.L)
        Ba = (ctypes.c_int32 * 4)(*self.block)
        h = ctypes.c_void_p()
        _check(lib().dw_field_create(ctx.handle, La, Ba, _dev_ptr(U), _stream(stream), ctypes.byref(h)),
               "dw_field_create")
        self.handle = h
        _live["field"].add(self)
        self.volume = int(lib().dw_field_volume(h))
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()

    def set_clover(self, csw: float, stream=None):
        """Add the clover term with coefficient csw (0 removes it); see dw_field_set_clover."""
        _check(lib().dw_field_set_clover(self.handle, float(csw), _stream(stream)), "dw_field_set_clover")
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        self.csw = float(csw)

    def close(self):
        if getattr(self, "handle", None):
            lib().dw_field_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers --------------------------------------------------------------
    def _nrhs(self, t):
        n = t.numel() // (self.volume * 12)
        if n * self.volume * 12 != t.numel():
            raise ValueError("spinor tensor size is not a multiple of the lattice volume * 12")
        return n

    def apply(self, m0: float, x: torch.Tensor, y: torch.Tensor | None = None, stream=None):
        """y = D x (eq. 1), FP64. Asynchronous on the stream."""
        if y is None:
            y = torch.empty_like(x)
        _check(lib().dw_apply(self.handle, float(m0), _dev_ptr(x), _dev_ptr(y), self._nrhs(x), _stream(stream)),
               "dw_apply")
        return y

    def apply_noalloc(self, m0: float, x: torch.Tensor, y: torch.Tensor, stream=None):
        """y = D x through dw_apply_noalloc (no device allocation; the caller
        provides y). Asynchronous on the stream."""
        _check(lib().dw_apply_noalloc(self.handle, float(m0), _dev_ptr(x), _dev_ptr(y), self._nrhs(x),
                                      _stream(stream)), "dw_apply_noalloc")
        return y

    def internal_bytes(self, prec, nrhs=1):
        return int(lib().dw_internal_bytes(self.handle, int(prec), int(nrhs)))

    def pack(self, prec, x: torch.Tensor, stream=None):
        nrhs = self._nrhs(x)
        out = torch.empty(self.internal_bytes(prec, nrhs), dtype=torch.uint8, device=x.device)
        _check(lib().dw_pack(self.handle, int(prec), _dev_ptr(x), _dev_ptr(out, None), nrhs, _stream(stream)),
               "dw_pack")
        return out

    def unpack(self, prec, xi: torch.Tensor, nrhs=1, stream=None):
        shp = (nrhs,) + tuple(reversed(self.L)) + (4, 3)
        out = torch.empty(shp, dtype=torch.complex128, device=xi.device)
        _check(lib().dw_unpack(self.handle, int(prec), _dev_ptr(xi, None), _dev_ptr(out), nrhs, _stream(stream)),
               "dw_unpack")
        return out

    def apply_ex(self, m0, prec, xi: torch.Tensor, yi: torch.Tensor, nrhs=1, stream=None):
        """y = D x on internal-layout buffers at precision prec (asynchronous)."""
        _check(lib().dw_apply_ex(self.handle, float(m0), int(prec), _dev_ptr(xi, None), _dev_ptr(yi, None),
                                 int(nrhs), _stream(stream)), "dw_apply_ex")

    def sap(self, m0: float, params: SapParams, v: torch.Tensor, z: torch.Tensor | None = None, stream=None):
        """z = M v: SAP (Alg. 2) with MR block solves. Asynchronous on the stream."""
        if z is None:
            z = torch.empty_like(v)
        p = params._c()
        _check(lib().sap_precondition(self.handle, float(m0), ctypes.byref(p), _dev_ptr(v), _dev_ptr(z),
                                      self._nrhs(v), _stream(stream)), "sap_precondition")
        return z

    def sap_solve(self, m0: float, params: SapParams, b: torch.Tensor, niter: int, x: torch.Tensor | None = None,
                  stream=None):
        """SAP as a stand-alone solver: x_{k+1} = x_k + M (b - D x_k) from x_0 = 0.
        Returns (x_niter, relative FP64 residuals for k = 0..niter). Synchronous."""
        if x is None:
            x = torch.empty_like(b)
        if self._nrhs(b) != 1:
            raise ValueError("sap_solve takes one right-hand side")
        p = params._c()
        res = (ctypes.c_double * (int(niter) + 1))()
        _check(lib().sap_solve(self.handle, float(m0), ctypes.byref(p), _dev_ptr(b), _dev_ptr(x), int(niter), res,
                               _stream(stream)), "sap_solve")
        return x, list(res)

    def solve(self, m0: float, params: SolverParams, b: torch.Tensor, x: torch.Tensor | None = None,
              stream=None, raise_on_notconv=True):
        """x = D^{-1} b by SAP-preconditioned FGMRES-DR (Alg. 4). Returns (x, [SolveStats])."""
        if x is None:
            x = torch.empty_like(b)
        nrhs = self._nrhs(b)
        st = (_Stats * nrhs)()
        p = params._c()
        status = lib().fgmresdr_solve(self.handle, float(m0), ctypes.byref(p), _dev_ptr(b), _dev_ptr(x), nrhs, st,
                                      _stream(stream))
        stats = [SolveStats(bool(s.converged), s.iterations, s.cycles, s.clean_restarts, s.true_relres,
                            s.implicit_relres, s.seconds) for s in st]
        if status == DW_ENOTCONV and not raise_on_notconv:
            return x, stats
        _check(status, "fgmresdr_solve")
        return x, stats


def _request(L, block, m0, U, b, x, params: SolverParams, csw=0.0):
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    if tuple(U.shape) != (4, Lt, Lz, Ly, Lx, 3, 3):
        raise ValueError(f"gauge shape {tuple(U.shape)} does not match L={tuple(L)}")
    vol12 = Lx * Ly * Lz * Lt * 12
    nrhs = b.numel() // vol12
    if nrhs * vol12 != b.numel() or x.numel() != b.numel():
        raise ValueError("b and x must hold a whole number of spinor fields of the lattice")
    r = _Request()
    for i in range(4):
        r.L[i], r.block[i] = (Lx, Ly, Lz, Lt)[i], int(block[i])
    r.m0, r.csw, r.nrhs, r.reserved = float(m0), float(csw), nrhs, 0
    r.U, r.b, r.x = _dev_ptr(U), _dev_ptr(b), _dev_ptr(x)
    r.params = params._c()
    return r


class Server:
    """Continuous-batching solve server: FIFO queue, footprint admission, slots on their own streams.

    submit() returns a ticket; poll() returns None while the request waits or
    runs, else (x, [SolveStats], times) and forgets the ticket. The server
    keeps the request's tensors alive until then. Inputs are read on the
    server's streams, so submit() first waits for the caller's stream.
    """

    def __init__(self, ctx: Context, slots: int = 2, queue_capacity: int = 64, budget_bytes: float = 0.0):
        p = _ServerParams(int(slots), int(queue_capacity), float(budget_bytes))
        h = ctypes.c_void_p()
        _check(lib().dw_server_create(ctx.handle, ctypes.byref(p), ctypes.byref(h)), "dw_server_create")
        self.ctx = ctx
        self.handle = h
        _live["server"].add(self)
        self._live = {}

    @staticmethod
    def footprint(L, block, m0, U, b, params: SolverParams, x=None, csw=0.0):
        r = _request(L, block, m0, U, b, b if x is None else x, params, csw)
        return int(lib().dw_request_footprint(ctypes.byref(r)))

    def submit(self, L, block, m0: float, U: torch.Tensor, b: torch.Tensor, params: SolverParams,
               x: torch.Tensor | None = None, csw: float = 0.0):
        if x is None:
            x = torch.empty_like(b)
        r = _request(L, block, m0, U, b, x, params, csw)
        torch.cuda.current_stream().synchronize()
        t = ctypes.c_uint64()
        _check(lib().solve_submit(self.handle, ctypes.byref(r), ctypes.byref(t)), "solve_submit")
        self._live[t.value] = (U, b, x, r.nrhs)
        return t.value

    def poll(self, ticket: int):
        U, b, x, nrhs = self._live[ticket]
        state = ctypes.c_int32()
        st = (_Stats * nrhs)()
        tm = _ReqTimes()
        _check(lib().solve_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(state), st, ctypes.byref(tm)),
               "solve_poll")
        if state.value in (REQ_QUEUED, REQ_RUNNING):
            return None
        del self._live[ticket]
        if state.value == REQ_FAILED:
            raise DwError(DW_EHIP, "request failed: " + lib().dw_last_error().decode(errors="replace"))
        stats = [SolveStats(bool(s.converged), s.iterations, s.cycles, s.clean_restarts, s.true_relres,
                            s.implicit_relres, s.seconds) for s in st]
        return x, stats, {"queued": tm.queued, "running": tm.running, "latency": tm.latency}

    def wait(self, ticket: int, poll_s: float = 1e-3):
        import time
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            time.sleep(poll_s)

    def close(self):
        if getattr(self, "handle", None):
            lib().dw_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class TuneSpace:
    """Search space of dw_autotune: block shapes (empty = the library's default
    set), MR steps and SAP cycles (inclusive ranges), (m, k) pairs."""
    blocks: tuple = ()
    nmr: tuple = (2, 8)
    s: tuple = (1, 4)
    mk: tuple = ()
    repeats: int = 1
    passes: int = 1
    iter_cap: float = 3.0

    def _c(self):
        t = _TuneSpace()
        if len(self.blocks) > 16 or len(self.mk) > 8:
            raise ValueError("at most 16 block shapes and 8 (m, k) pairs")
        t.nblocks = len(self.blocks)
        for i, B in enumerate(self.blocks):
            for j in range(4):
                t.blocks[i][j] = int(B[j])
        t.nmr_min, t.nmr_max = int(self.nmr[0]), int(self.nmr[1])
        t.s_min, t.s_max = int(self.s[0]), int(self.s[1])
        t.nmk = len(self.mk)
        for i, (m, k) in enumerate(self.mk):
            t.mk[i][0], t.mk[i][1] = int(m), int(k)
        t.repeats, t.passes, t.iter_cap = int(self.repeats), int(self.passes), float(self.iter_cap)
        return t


def _params_from_c(p: _SolverParams) -> SolverParams:
    return SolverParams(m=p.m, k=p.k, max_iter=p.max_iter, tol=p.tol, restart_t=p.restart_t,
                        sap=SapParams(block=tuple(p.sap.block), ncycles=p.sap.ncycles, nmr=p.sap.nmr,
                                      storage=p.sap.storage, mr_reduction=p.sap.mr_reduction),
                        shared_defl=p.shared_defl, flags=p.flags)


class TuneCache:
    """JSON file of tuned solver parameters, keyed by device architecture,
    lattice, mass, storage precision, RHS count and tolerance."""

    def __init__(self, path: str):
        self.path = path

    @staticmethod
    def key(arch, L, m0, base: SolverParams, nrhs):
        return (f"{arch}|L={'x'.join(str(int(v)) for v in L)}|m0={float(m0):.6f}|prec={base.sap.storage}"
                f"|nrhs={int(nrhs)}|tol={float(base.tol):.3g}")

    def _load(self):
        import json
        if not os.path.exists(self.path):
            return {}
        with open(self.path) as fh:
            return json.load(fh)

    def get(self, key):
        e = self._load().get(key)
        if e is None:
            return None
        p = e["params"]
        return SolverParams(m=p["m"], k=p["k"], max_iter=p["max_iter"], tol=p["tol"], restart_t=p["restart_t"],
                            sap=SapParams(block=tuple(p["block"]), ncycles=p["ncycles"], nmr=p["nmr"],
                                          storage=p["storage"], mr_reduction=p.get("mr_reduction", 0.0)))

    def put(self, key, params: SolverParams, trials=()):
        import json
        d = self._load()
        d[key] = {"params": {"m": params.m, "k": params.k, "max_iter": params.max_iter, "tol": params.tol,
                             "restart_t": params.restart_t, "block": list(params.sap.block),
                             "ncycles": params.sap.ncycles, "nmr": params.sap.nmr, "storage": params.sap.storage,
                             "mr_reduction": params.sap.mr_reduction},
                  "trials": [dict(t) for t in trials]}
        tmp = self.path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(d, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def autotune(ctx: Context, L, U: torch.Tensor, m0: float, base: SolverParams, b: torch.Tensor,
             space: TuneSpace | None = None, cache: TuneCache | None = None, max_trials: int = 64, stream=None,
             csw: float = 0.0):
    """Tune (block, nmr, s, m, k) by time to solution (dw_autotune). Returns
    (best SolverParams, list of trial dicts); with a cache, a stored result is
    returned without solving (trials then empty)."""
    space = space or TuneSpace()
    vol12 = int(L[0]) * int(L[1]) * int(L[2]) * int(L[3]) * 12
    nrhs = b.numel() // vol12
    if nrhs * vol12 != b.numel() or nrhs < 1:
        raise ValueError("b must hold a whole number of spinor fields of the lattice")
    key = None
    if cache is not None:
        arch = torch.cuda.get_device_properties(b.device).gcnArchName
        key = TuneCache.key(arch, L, m0, base, nrhs) + (f"|csw={float(csw):.6f}" if csw else "")
        hit = cache.get(key)
        if hit is not None:
            return hit, []
    La = (ctypes.c_int32 * 4)(*(int(v) for v in L))
    x = torch.empty_like(b)
    tr = (_TuneTrial * int(max_trials))()
    nt = ctypes.c_int32()
    best = _SolverParams()
    bp, sp = base._c(), space._c()
    _check(lib().dw_autotune(ctx.handle, La, _dev_ptr(U), float(m0), float(csw), ctypes.byref(bp), ctypes.byref(sp),
                             _dev_ptr(b), _dev_ptr(x), nrhs, tr, int(max_trials), ctypes.byref(nt),
                             ctypes.byref(best), _stream(stream)), "dw_autotune")
    trials = []
    for t in tr[:nt.value]:
        p = t.params
        trials.append({"block": list(p.sap.block), "nmr": p.sap.nmr, "ncycles": p.sap.ncycles, "m": p.m,
                       "k": p.k, "converged": bool(t.converged), "iterations": t.iterations,
                       "seconds": t.seconds})
    bestp = _params_from_c(best)
    if cache is not None:
        cache.put(key, bestp, trials)
    return bestp, trials


def _host_c128(a):
    import numpy as np
    return np.asfortranarray(np.asarray(a, dtype=np.complex128))


def dense_lsq(ctx: Context, Hhat, c):
    """eta = argmin ||c - H^ eta|| by the solver's small dense kernel (Section 4.2).
    Hhat: (cols + 1) x cols, c: cols + 1 (host arrays). Returns (eta, residual norm)."""
    import numpy as np
    H = _host_c128(Hhat)
    cols = H.shape[1]
    if H.shape[0] != cols + 1:
        raise ValueError("H^ must have one more row than columns")
    cv = np.ascontiguousarray(np.asarray(c, dtype=np.complex128).reshape(-1))
    eta = np.zeros(cols, dtype=np.complex128)
    res = ctypes.c_double()
    _check(lib().dw_dense_lsq(ctx.handle, int(cols), H.ctypes.data, cv.ctypes.data, eta.ctypes.data,
                              ctypes.byref(res)), "dw_dense_lsq")
    return eta, res.value


def dense_restart(ctx: Context, Hhat, c, eta, k: int):
    """The deflated-restart step (Lemma 1, Section 4.4) by the solver's small dense kernel.
    Returns (harmonic Ritz values sorted by modulus, Q_{k+1}, H^_k, status)."""
    import numpy as np
    H = _host_c128(Hhat)
    mm = H.shape[1]
    if H.shape[0] != mm + 1:
        raise ValueError("H^ must have one more row than columns")
    cv = np.ascontiguousarray(np.asarray(c, dtype=np.complex128).reshape(-1))
    ev = np.ascontiguousarray(np.asarray(eta, dtype=np.complex128).reshape(-1))
    ritz = np.zeros(mm, dtype=np.complex128)
    Q = np.zeros((mm + 1, k + 1), dtype=np.complex128, order="F")
    Hk = np.zeros((k + 1, k), dtype=np.complex128, order="F")
    status = ctypes.c_int32()
    _check(lib().dw_dense_restart(ctx.handle, int(mm), int(k), H.ctypes.data, cv.ctypes.data, ev.ctypes.data,
                                  ritz.ctypes.data, Q.ctypes.data, Hk.ctypes.data, ctypes.byref(status)),
           "dw_dense_restart")
    return ritz, np.asarray(Q), np.asarray(Hk), int(status.value)


def to_device(a, device="cuda"):
    """numpy complex array -> contiguous complex128 tensor on the GPU."""
    import numpy as np
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(device)
