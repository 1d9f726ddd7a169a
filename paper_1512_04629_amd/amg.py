"""Python binding of libamg355 (the C ABI declared in include/amg.h).

Argument marshalling only: every step of setup upload, sparsification and
solve runs in the library.  Device arrays are torch CUDA tensors (float64,
contiguous); device memory owned by the library comes from PyTorch's caching
allocator through the ABI's allocator callback, and all work is issued on
the torch stream current when the hierarchy is created.

The library must be built (``python -m paper_1512_04629_amd.build``); there is
no fallback path: loading fails loudly if the shared object is missing.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libamg355.so")

OK, NOTHING_TO_REINTRODUCE, NOT_READY = 0, 1, 2
STATIONARY, PCG = 0, 1
MAT = {"A": 0, "AHAT": 1, "P": 2, "R": 3}
MASK = {"M": 0, "KEEP": 1}
VEC = {"ROWMAX": 0, "DINV": 1}
OP = {"RESIDUAL": 0, "JACOBI": 1, "RESTRICT": 2, "INTERPOLATE": 3, "COARSE_SOLVE": 4,
      "SPMV_A": 5, "SPMV_AHAT": 6, "GS_FORWARD": 7, "GS_BACKWARD": 8}
KERNEL = {"JACOBI": 0, "JACOBI_ZERO": 1, "RESIDUAL": 2, "RESTRICT": 3, "INTERP": 4,
          "COARSE": 5, "SPMV_DOT": 6, "VECTOR": 7, "SPARSIFY": 8, "LUMP_DEN": 9,
          "LUMP_SHARES": 10}

# every symbol include/amg.h declares
ABI_SYMBOLS = (
    "amg_setup_params_default", "amg_solve_params_default", "amg_setup_from_csr",
    "amg_setup_nongalerkin_from_csr", "amg_setup_device", "amg_setup_profile_enable", "amg_setup_profile_read",
    "amg_sparsify", "amg_sparsify_levels", "amg_set_method", "amg_set_relaxation", "amg_set_lumping", "amg_set_lump_shapes", "amg_reintroduce", "amg_solve", "amg_solve_noalloc", "amg_vcycle",
    "amg_vcycle32",
    "amg_solve_block", "amg_vcycle_block", "amg_vcycle_block32", "amg_batch_bytes", "amg_batch_create",
    "amg_batch_submit", "amg_batch_step", "amg_batch_poll", "amg_batch_collect", "amg_batch_slots",
    "amg_batch_destroy", "amg_device_bytes", "amg_level_op", "amg_num_levels", "amg_get_level", "amg_export_level", "amg_export_mask",
    "amg_export_vector", "amg_export_split", "amg_set_compact_indices", "amg_index_width", "amg_row_format",
    "amg_profile_enable", "amg_profile_read",
    "amg_destroy", "amg_status_string", "amg_last_error",
)


COARSENINGS = {"rs": 0, "pmis": 1}     # AMG_COARSEN_RS, AMG_COARSEN_PMIS
SETUP_KERNELS = ("STRENGTH", "SPLIT", "INTERP", "TRANSPOSE", "EXPAND", "SORT", "COMBINE", "SYMMETRIZE")


def setup_profile_enable(on: bool = True):
    """Starts (resetting the totals) or stops the process-wide timing of the
    device setup's kernel classes."""
    load_library().amg_setup_profile_enable(int(bool(on)))


def setup_profile_read() -> dict:
    """{class: (timed groups, milliseconds, algorithmic bytes)} since the last enable."""
    lib = load_library()
    out = {}
    for k, name in enumerate(SETUP_KERNELS):
        c, ms, nb = C.c_int64(), C.c_double(), C.c_double()
        st = lib.amg_setup_profile_read(k, C.byref(c), C.byref(ms), C.byref(nb))
        if st != OK:
            raise AmgError(st, lib.amg_status_string(st).decode())
        out[name] = (c.value, ms.value, nb.value)
    return out


class AmgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class SetupParams(C.Structure):
    _fields_ = [("theta", C.c_double), ("max_coarse", C.c_int32), ("max_levels", C.c_int32),
                ("omega", C.c_double), ("nu_pre", C.c_int32), ("nu_post", C.c_int32)]


class SolveParams(C.Structure):
    _fields_ = [("method", C.c_int32), ("rtol", C.c_double), ("maxit", C.c_int32),
                ("adaptive", C.c_int32), ("k", C.c_int32), ("s", C.c_int32),
                ("rho_max", C.c_double), ("gamma_min", C.c_double), ("precision", C.c_int32),
                ("zero_guess", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("reintroductions", C.c_int32),
                ("converged", C.c_int32), ("relres", C.c_double), ("rho_avg", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)

_lib = None


def load_library():
    """Loads libamg355.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1512_04629_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    lib.amg_setup_params_default.argtypes = [P(SetupParams)]
    lib.amg_solve_params_default.argtypes = [P(SolveParams)]
    lib.amg_setup_from_csr.argtypes = [i64, vp, vp, vp, P(SetupParams), vp, ALLOC_FN, FREE_FN, vp, P(vp)]
    lib.amg_setup_nongalerkin_from_csr.argtypes = [i64, vp, vp, vp, P(SetupParams), vp, i32, vp, ALLOC_FN,
                                                   FREE_FN, vp, P(vp)]
    lib.amg_setup_device.argtypes = [i64, i64, vp, vp, vp, P(SetupParams), i32, C.c_uint64, vp, ALLOC_FN,
                                     FREE_FN, vp, P(vp)]
    lib.amg_setup_profile_enable.argtypes = [i32]
    lib.amg_setup_profile_read.argtypes = [i32, P(i64), P(f64), P(f64)]
    lib.amg_sparsify.argtypes = [vp, f64, i32]
    lib.amg_sparsify_levels.argtypes = [vp, vp, i32]
    lib.amg_reintroduce.argtypes = [vp, i32, f64, P(i32)]
    lib.amg_set_method.argtypes = [vp, i32]
    lib.amg_set_relaxation.argtypes = [vp, i32, i32]
    lib.amg_set_lumping.argtypes = [vp, i32]
    lib.amg_set_lump_shapes.argtypes = [vp, f64, f64, i32]
    lib.amg_solve.argtypes = [vp, vp, vp, P(SolveParams), P(SolveInfo), vp]
    lib.amg_solve_noalloc.argtypes = [vp, vp, vp, P(SolveParams), P(SolveInfo), vp]
    lib.amg_vcycle.argtypes = [vp, vp, vp]
    lib.amg_vcycle32.argtypes = [vp, vp, vp]
    lib.amg_solve_block.argtypes = [vp, i32, vp, vp, P(SolveParams), P(SolveInfo), vp, vp]
    lib.amg_vcycle_block.argtypes = [vp, i32, vp, vp]
    lib.amg_vcycle_block32.argtypes = [vp, i32, vp, vp]
    lib.amg_batch_bytes.argtypes = [vp, i32, i32, P(i64)]
    lib.amg_batch_create.argtypes = [vp, i32, i32, f64, i32, i32, P(vp)]
    lib.amg_batch_submit.argtypes = [vp, vp, P(i32)]
    lib.amg_batch_step.argtypes = [vp, i32, P(i32)]
    lib.amg_batch_poll.argtypes = [vp, i32, vp]
    lib.amg_batch_collect.argtypes = [vp, i32, vp, P(i32), P(f64), P(i32)]
    lib.amg_batch_slots.argtypes = [vp, vp]
    lib.amg_batch_destroy.argtypes = [vp]
    lib.amg_batch_destroy.restype = None
    lib.amg_device_bytes.argtypes = [vp, P(i64)]
    lib.amg_level_op.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.amg_num_levels.argtypes = [vp, P(i32)]
    lib.amg_get_level.argtypes = [vp, i32, P(i64), P(i64), P(i64), P(i64), P(i64), P(f64), P(i64)]
    lib.amg_export_level.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.amg_export_mask.argtypes = [vp, i32, i32, vp]
    lib.amg_export_vector.argtypes = [vp, i32, i32, vp]
    lib.amg_export_split.argtypes = [vp, i32, vp]
    lib.amg_set_compact_indices.argtypes = [vp, i32]
    lib.amg_index_width.argtypes = [vp, i32, i32, P(i32)]
    lib.amg_row_format.argtypes = [vp, i32, i32, P(i32)]
    lib.amg_profile_enable.argtypes = [vp, i32, i32, i32]
    lib.amg_profile_read.argtypes = [vp, i32, i32, P(i64), P(f64)]
    lib.amg_destroy.argtypes = [vp]
    lib.amg_destroy.restype = None
    lib.amg_status_string.argtypes = [C.c_int]
    lib.amg_status_string.restype = C.c_char_p
    lib.amg_last_error.argtypes = [vp]
    lib.amg_last_error.restype = C.c_char_p
    for name in ("amg_setup_from_csr", "amg_setup_nongalerkin_from_csr", "amg_setup_device",
                 "amg_setup_profile_enable", "amg_setup_profile_read", "amg_sparsify", "amg_sparsify_levels", "amg_set_method",
                 "amg_set_relaxation", "amg_set_lumping", "amg_set_lump_shapes", "amg_reintroduce",
                 "amg_solve", "amg_solve_noalloc", "amg_vcycle", "amg_vcycle32", "amg_solve_block", "amg_vcycle_block",
                 "amg_vcycle_block32", "amg_batch_bytes", "amg_batch_create", "amg_batch_submit",
                 "amg_batch_step", "amg_batch_poll", "amg_batch_collect", "amg_batch_slots", "amg_device_bytes",
                 "amg_level_op", "amg_num_levels", "amg_get_level",
                 "amg_export_level", "amg_export_mask", "amg_export_vector", "amg_export_split",
                 "amg_set_compact_indices", "amg_index_width", "amg_row_format", "amg_profile_enable",
                 "amg_profile_read"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libamg355 needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


_torch_mem = {}


@C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
def _torch_alloc(nbytes, stream, user):
    try:
        if not _torch_mem:
            import torch
            _torch_mem["alloc"] = torch.cuda.caching_allocator_alloc
            _torch_mem["free"] = torch.cuda.caching_allocator_delete
        return _torch_mem["alloc"](int(nbytes), stream=int(stream or 0))
    except Exception:       # reported to the library as NULL -> out of memory
        return None


@C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
def _torch_free(ptr, nbytes, stream, user):
    free = _torch_mem.get("free")
    if ptr and free is not None:
        try:
            free(int(ptr))
        except Exception:   # interpreter shutdown: the process releases the memory
            pass


_live = weakref.WeakSet()


@atexit.register
def _close_all():
    """Destroys the handles still alive before the interpreter tears torch down."""
    for h in list(_live):
        try:
            h.close()
        except Exception:
            pass


@dataclass
class BlockSolveResult:
    status: int
    iters: int
    converged: bool
    relres: float
    col_iters: np.ndarray
    col_relres: np.ndarray


@dataclass
class SolveResult:
    status: int
    iters: int
    restarts: int
    reintroductions: int
    converged: bool
    relres: float
    rho_avg: float
    hist: np.ndarray


def _dptr(t, n=None, name="array"):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return C.c_void_p(t.data_ptr())


class Hierarchy:
    """A device-resident AMG hierarchy (one amg_handle)."""

    def __init__(self, A, theta=0.25, max_coarse=49, max_levels=25, omega=2.0 / 3.0,
                 nu_pre=1, nu_post=1, torch_allocator=True, nongalerkin_gamma=None, setup="host",
                 coarsening="rs", seed=0):
        """nongalerkin_gamma: per-level tolerances of the method of non-Galerkin
        coarse grids (each coarse product sparsified during setup); None for
        the Galerkin hierarchy.

        setup="device": the hierarchy is built by amg_setup_device from device
        copies of A (or from A itself when it is a tuple (n, row_ptr, col, val)
        of CUDA tensors), with coarsening "rs" (the same hierarchy as the host
        setup) or "pmis" (weights of level l from the SplitMix64 stream
        seed + l)."""
        if setup not in ("host", "device") or coarsening not in COARSENINGS:
            raise ValueError(f"unknown setup {setup!r} or coarsening {coarsening!r}")
        if setup == "host" and coarsening != "rs":
            raise ValueError("PMIS coarsening runs in the device setup only")
        if setup == "device" and nongalerkin_gamma is not None:
            raise ValueError("the device setup builds the Galerkin hierarchy")
        torch = _torch()
        lib = load_library()
        self._lib = lib
        sp = SetupParams(float(theta), int(max_coarse), int(max_levels), float(omega),
                         int(nu_pre), int(nu_post))
        self.stream = torch.cuda.current_stream()
        h = C.c_void_p()
        alloc = _torch_alloc if torch_allocator else ALLOC_FN()
        free = _torch_free if torch_allocator else FREE_FN()
        if setup == "device":
            if isinstance(A, tuple):
                n, rp_d, ci_d, v_d = A
            else:
                n = A.n
                rp_d = torch.from_numpy(np.ascontiguousarray(A.row_ptr, np.int32)).cuda()
                ci_d = torch.from_numpy(np.ascontiguousarray(A.col, np.int32)).cuda()
                v_d = torch.from_numpy(np.ascontiguousarray(A.val, np.float64)).cuda()
            if (rp_d.dtype != torch.int32 or ci_d.dtype != torch.int32 or v_d.dtype != torch.float64
                    or not (rp_d.is_cuda and ci_d.is_cuda and v_d.is_cuda)):
                raise ValueError("device CSR: int32 row_ptr and col, float64 values, CUDA tensors")
            self.n = int(n)
            st = lib.amg_setup_device(self.n, int(ci_d.numel()), rp_d.data_ptr(), ci_d.data_ptr(),
                                      v_d.data_ptr(), C.byref(sp), COARSENINGS[coarsening],
                                      int(seed) & 0xFFFFFFFFFFFFFFFF, C.c_void_p(self.stream.cuda_stream),
                                      alloc, free, None, C.byref(h))
            if st != OK:
                raise AmgError(st, lib.amg_last_error(None).decode())
            self._finish(h)
            return
        self.n = int(A.n)
        rp = np.ascontiguousarray(A.row_ptr, np.int32)
        ci = np.ascontiguousarray(A.col, np.int32)
        v = np.ascontiguousarray(A.val, np.float64)
        if nongalerkin_gamma is None:
            st = lib.amg_setup_from_csr(self.n, rp.ctypes.data, ci.ctypes.data, v.ctypes.data,
                                        C.byref(sp), C.c_void_p(self.stream.cuda_stream), alloc, free,
                                        None, C.byref(h))
        else:
            ng = np.ascontiguousarray(nongalerkin_gamma, np.float64)
            st = lib.amg_setup_nongalerkin_from_csr(self.n, rp.ctypes.data, ci.ctypes.data, v.ctypes.data,
                                                    C.byref(sp), ng.ctypes.data, len(ng),
                                                    C.c_void_p(self.stream.cuda_stream), alloc, free, None,
                                                    C.byref(h))
        if st != OK:
            raise AmgError(st, lib.amg_last_error(None).decode())
        self._finish(h)

    def _finish(self, h):
        self._h = h
        _live.add(self)
        nl = C.c_int32()
        self._check(self._lib.amg_num_levels(h, C.byref(nl)))
        self.nlev = nl.value

    # -- plumbing --------------------------------------------------------
    def _check(self, st, allowed=(OK,)):
        if st not in allowed:
            raise AmgError(st, self._lib.amg_last_error(self._h).decode() or
                           self._lib.amg_status_string(st).decode())
        return st

    def close(self):
        b = getattr(self, "_batch", None)
        if b is not None:
            b.close()
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.amg_destroy(h)
        self._h = None

    def device_bytes(self) -> int:
        v = C.c_int64()
        self._check(self._lib.amg_device_bytes(self._h, C.byref(v)))
        return v.value

    def batch_bytes(self, slots=16, precision=32) -> int:
        v = C.c_int64()
        self._check(self._lib.amg_batch_bytes(self._h, int(slots), int(precision), C.byref(v)))
        return v.value

    def batch(self, slots=16, precision=32, tol=1e-10, maxit=300, graphs=True) -> "Batch":
        """The continuous-batching engine of this hierarchy (at most one)."""
        return Batch(self, slots, precision, tol, maxit, graphs)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- sparsification ------------------------------------------------------
    def sparsify(self, gamma: float, first_level: int = 2):
        self._check(self._lib.amg_sparsify(self._h, float(gamma), int(first_level)))

    def sparsify_levels(self, gammas):
        g = np.ascontiguousarray(gammas, np.float64)
        self._check(self._lib.amg_sparsify_levels(self._h, g.ctypes.data, len(g)))

    def set_method(self, hybrid: bool) -> None:
        """Sparse Galerkin (False, default) or Hybrid Galerkin (True) for later
        sparsify / reintroduce calls."""
        self._check(self._lib.amg_set_method(self._h, 1 if hybrid else 0))

    def reintroduce(self, s: int = 1, gamma_min: float = 0.01):
        first = C.c_int32(-1)
        st = self._check(self._lib.amg_reintroduce(self._h, int(s), float(gamma_min), C.byref(first)),
                         allowed=(OK, NOTHING_TO_REINTRODUCE))
        return st, first.value

    # -- solve -------------------------------------------------------------
    def solve(self, b, x, method=PCG, tol=1e-8, maxit=200, adaptive=False, k=3, s=1,
              rho_max=0.5, gamma_min=0.01, precision=64, raise_on_error=False, noalloc=False,
              zero_guess=False) -> SolveResult:
        """precision=32 runs the V-cycle in FP32 inside the FP64 iteration.
        noalloc=True calls amg_solve_noalloc (work memory in the library's
        static device array; FP64 only, n <= 2,097,152).  zero_guess=True
        starts from x0 = 0 whatever x holds (x is zeroed, r0 = b)."""
        p = SolveParams(int(method), float(tol), int(maxit), int(bool(adaptive)), int(k), int(s),
                        float(rho_max), float(gamma_min), int(precision), int(bool(zero_guess)))
        info = SolveInfo()
        hist = np.full(maxit + 1, np.nan)
        fn = self._lib.amg_solve_noalloc if noalloc else self._lib.amg_solve
        st = fn(self._h, _dptr(b, self.n, "b"), _dptr(x, self.n, "x"), C.byref(p), C.byref(info),
                hist.ctypes.data)
        if st not in (OK, -5, -6) or raise_on_error:
            self._check(st)
        return SolveResult(st, info.iters, info.restarts, info.reintroductions, bool(info.converged),
                           info.relres, info.rho_avg, hist[: info.iters + 1].copy())

    def vcycle(self, b, x):
        self._check(self._lib.amg_vcycle(self._h, _dptr(b, self.n, "b"), _dptr(x, self.n, "x")))

    def vcycle32(self, b, x):
        """One FP32 V-cycle x <- V32(b, x) on float32 CUDA tensors."""
        torch = _torch()
        for t, name in ((b, "b"), (x, "x")):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
                    and t.is_contiguous() and t.numel() == self.n):
                raise TypeError(f"{name} must be a contiguous float32 CUDA tensor of {self.n} entries")
        self._check(self._lib.amg_vcycle32(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr())))

    def _block(self, t, name, dtype, nrhs=None):
        torch = _torch()
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()
                and t.dim() == 2 and t.shape[0] == self.n and (nrhs is None or t.shape[1] == nrhs)):
            raise TypeError(f"{name} must be a contiguous {dtype} CUDA tensor of shape ({self.n}, nrhs)")
        return C.c_void_p(t.data_ptr())

    def solve_block(self, b, x, method=PCG, tol=1e-10, maxit=200, precision=32,
                    raise_on_error=False) -> BlockSolveResult:
        """Solves all columns of the (n, nrhs) float64 blocks b, x at once: PCG
        per column, or (method=STATIONARY) iterative refinement; precision=32
        runs the V-cycle in FP32."""
        torch = _torch()
        nrhs = int(b.shape[1]) if b.dim() == 2 else 0
        pb, px = self._block(b, "b", torch.float64), self._block(x, "x", torch.float64, nrhs)
        p = SolveParams(int(method), float(tol), int(maxit), 0, 3, 1, 0.5, 0.01, int(precision))
        info = SolveInfo()
        ci = np.full(max(nrhs, 1), -2, np.int32)
        cr = np.full(max(nrhs, 1), np.nan)
        st = self._lib.amg_solve_block(self._h, nrhs, pb, px, C.byref(p), C.byref(info),
                                       ci.ctypes.data, cr.ctypes.data)
        if st not in (OK, -5, -6) or raise_on_error:
            self._check(st)
        return BlockSolveResult(st, info.iters, bool(info.converged), info.relres, ci[:nrhs].copy(),
                                cr[:nrhs].copy())

    def vcycle_block(self, b, x):
        """One V-cycle X <- V(B, X) on (n, 4|8|16) blocks, float64 or float32."""
        torch = _torch()
        fn = self._lib.amg_vcycle_block if b.dtype == torch.float64 else self._lib.amg_vcycle_block32
        nrhs = int(b.shape[1]) if b.dim() == 2 else 0
        self._check(fn(self._h, nrhs, self._block(b, "b", b.dtype), self._block(x, "x", b.dtype, nrhs)))

    def level_op(self, level: int, op: str, inp=None, x=None, out=None):
        args = [C.c_void_p(t.data_ptr()) if t is not None else None for t in (inp, x, out)]
        for t, name in ((inp, "in"), (x, "x"), (out, "out")):
            if t is not None:
                _dptr(t, None, name)
        self._check(self._lib.amg_level_op(self._h, int(level), OP[op], *args))

    # -- inspection ---------------------------------------------------------
    def level_info(self, l: int) -> dict:
        vals = [C.c_int64() for _ in range(5)]
        g = C.c_double()
        by = C.c_int64()
        self._check(self._lib.amg_get_level(self._h, int(l), *[C.byref(v) for v in vals],
                                            C.byref(g), C.byref(by)))
        n, nnz, nnz_hat, nnz_p, nc = (v.value for v in vals)
        return dict(n=n, nnz=nnz, nnz_hat=nnz_hat, nnz_P=nnz_p, n_coarse=nc, gamma=g.value,
                    bytes=by.value)

    def export(self, l: int, which: str):
        s = self.level_info(l)
        if which in ("A", "AHAT"):
            nr, nc, nnz = s["n"], s["n"], s["nnz"] if which == "A" else s["nnz_hat"]
        elif which == "P":
            nr, nc, nnz = s["n"], s["n_coarse"], s["nnz_P"]
        else:
            nr, nc, nnz = s["n_coarse"], s["n"], s["nnz_P"]
        rp = np.zeros(nr + 1, np.int32)
        ci = np.zeros(max(nnz, 1), np.int32)
        v = np.zeros(max(nnz, 1), np.float64)
        self._check(self._lib.amg_export_level(self._h, int(l), MAT[which], rp.ctypes.data,
                                               ci.ctypes.data, v.ctypes.data))
        return nr, nc, rp, ci[:nnz].copy(), v[:nnz].copy()

    def mask(self, l: int, which: str) -> np.ndarray:
        nnz = self.level_info(l)["nnz"]
        out = np.zeros(max(nnz, 1), np.uint8)
        self._check(self._lib.amg_export_mask(self._h, int(l), MASK[which], out.ctypes.data))
        return out[:nnz]

    def vector(self, l: int, which: str) -> np.ndarray:
        out = np.zeros(self.level_info(l)["n"], np.float64)
        self._check(self._lib.amg_export_vector(self._h, int(l), VEC[which], out.ctypes.data))
        return out

    def split(self, l: int) -> np.ndarray:
        out = np.zeros(self.level_info(l)["n"], np.int32)
        self._check(self._lib.amg_export_split(self._h, int(l), out.ctypes.data))
        return out

    def set_lumping(self, mode: str = "diagonal"):
        """Where later sparsify / reintroduce calls put dropped entries:
        "diagonal" (Algorithm 3b) or "strong" (strong neighbours, Algorithm 3)."""
        if mode not in ("diagonal", "strong"):
            raise ValueError(f"unknown lumping {mode!r}")
        self._check(self._lib.amg_set_lumping(self._h, {"diagonal": 0, "strong": 1}[mode]))

    def set_lump_shapes(self, wide_mean_row: float = 0.0, den_wave_mean_row: float = -1.0,
                        small_rows: int = 4096):
        """Testing hook: launch shapes of the strong-lumping kernels (the same
        bits every way); the defaults are the library's."""
        self._check(self._lib.amg_set_lump_shapes(self._h, float(wide_mean_row), float(den_wave_mean_row),
                                                  int(small_rows)))

    def set_relaxation(self, kind: str = "jacobi", block_rows: int = 64):
        """Weighted Jacobi (default) or hybrid symmetric Gauss-Seidel with blocks
        of block_rows rows for later V-cycles and FP64 solves."""
        self._check(self._lib.amg_set_relaxation(self._h, {"jacobi": 0, "hybrid_gs": 1}[kind], int(block_rows)))

    def set_compact_indices(self, on: bool = True):
        """Builds (default) or drops the 16-bit column indices of A_l, P_l, R_l."""
        self._check(self._lib.amg_set_compact_indices(self._h, int(bool(on))))

    def row_format(self, l: int, which: str) -> str:
        """FP64 row kernel of matrix `which` of level l: "row", "stream" or "sell"."""
        f = C.c_int32()
        self._check(self._lib.amg_row_format(self._h, int(l), MAT[which], C.byref(f)))
        return ("row", "stream", "sell")[f.value]

    def index_width(self, l: int, which: str) -> int:
        """Bytes per column index the row kernels read for matrix `which` of level l."""
        b = C.c_int32()
        self._check(self._lib.amg_index_width(self._h, int(l), MAT[which], C.byref(b)))
        return b.value

    def gamma(self, l: int) -> float:
        return self.level_info(l)["gamma"]

    def bytes_per_cycle(self) -> int:
        return sum(self.level_info(l)["bytes"] for l in range(self.nlev))

    # -- kernel timing ---------------------------------------------------------
    def profile_enable(self, on: bool = True, kernel: str | None = None, level: int = -1):
        """Times launches of one kernel class (None: all) on one level (-1: all)."""
        kc = -1 if kernel is None else KERNEL[kernel]
        self._check(self._lib.amg_profile_enable(self._h, int(bool(on)), kc, int(level)))

    def profile_read(self, kernel: str, level: int):
        cnt = C.c_int64()
        ms = C.c_double()
        self._check(self._lib.amg_profile_read(self._h, KERNEL[kernel], int(level), C.byref(cnt),
                                               C.byref(ms)))
        return cnt.value, ms.value


class Batch:
    """Continuous-batching engine on one hierarchy (amg_batch): up to `slots`
    right-hand sides are solved together by PCG and a finished slot takes a
    new right-hand side at the next step."""

    FREE, SUBMITTED, ITERATING, FINISHED = 0, 1, 2, 3

    def __init__(self, hier: Hierarchy, slots=16, precision=32, tol=1e-10, maxit=300, graphs=True):
        if getattr(hier, "_batch", None) is not None:
            raise AmgError(-7, "the hierarchy already has a batch engine")
        self._lib = hier._lib
        self.hier = hier
        self.slots = int(slots)
        self.precision = int(precision)
        b = C.c_void_p()
        hier._check(self._lib.amg_batch_create(hier._h, self.slots, self.precision, float(tol), int(maxit),
                                               1 if graphs else 0, C.byref(b)))
        self._b = b
        hier._batch = self
        self._fin = np.zeros(self.slots, np.int32)

    def _check(self, st, allowed=(OK,)):
        return self.hier._check(st, allowed)

    def close(self):
        b = getattr(self, "_b", None)
        if b is not None and b.value:
            self._lib.amg_batch_destroy(b)
        self._b = None
        if getattr(self.hier, "_batch", None) is self:
            self.hier._batch = None

    def submit(self, rhs) -> int:
        """Copies rhs (float64 CUDA tensor of n entries) into a free slot.  The
        copy runs on the engine's stream: work that produced rhs on another
        stream must be ordered before it (e.g. engine_stream.wait_stream)."""
        slot = C.c_int32(-1)
        self._check(self._lib.amg_batch_submit(self._b, _dptr(rhs, self.hier.n, "rhs"), C.byref(slot)))
        return slot.value

    def step(self, iters: int = 1) -> bool:
        """Enqueues `iters` iterations of every active slot; False if there was
        no work."""
        launched = C.c_int32(0)
        self._check(self._lib.amg_batch_step(self._b, int(iters), C.byref(launched)))
        return bool(launched.value)

    def poll(self, wait=True):
        """Completes the last step: the list of slots that finished in it, or
        None (wait=False) while it is still running."""
        st = self._check(self._lib.amg_batch_poll(self._b, int(bool(wait)), self._fin.ctypes.data),
                         allowed=(OK, NOT_READY))
        if st == NOT_READY:
            return None
        return [int(c) for c in np.nonzero(self._fin)[0]]

    def collect(self, slot: int, x):
        """Copies a finished slot's solution into x (float64 CUDA tensor, on the
        hierarchy's stream) and frees the slot: (iterations, relres, status).
        Earlier writes to x on other streams must be ordered before this call,
        and later readers on other streams must wait for the engine's stream."""
        it, rr, st = C.c_int32(), C.c_double(), C.c_int32()
        self._check(self._lib.amg_batch_collect(self._b, int(slot), _dptr(x, self.hier.n, "x"), C.byref(it),
                                                C.byref(rr), C.byref(st)))
        return it.value, rr.value, st.value

    def states(self) -> np.ndarray:
        out = np.zeros(self.slots, np.int32)
        self._check(self._lib.amg_batch_slots(self._b, out.ctypes.data))
        return out
