"""ctypes front end of the C oracle (``amg_oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle is the plain FP64 CPU reference the
device library is checked against.  Only the tests, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py`` may import this module.  It shares no
code with the device library; the only common input is the seeded problem
generator module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "amg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# timing build of the CPU baseline: the same source with OpenMP row loops
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")

CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

STATIONARY, PCG = 0, 1
OK, NOTHING, EINVAL, EMATRIX, ENOMEM, ENOTCONV, EBREAK = 0, 1, -1, -2, -3, -5, -6
WHICH = {"A": 0, "AHAT": 1, "P": 2, "R": 3, "S": 4}


def build(force: bool = True, parallel: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction): the single-threaded
    parity build, or with parallel=True the OpenMP timing build (same bits)."""
    lib = LIB_OMP if parallel else LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(SRC):
        tmp = lib + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, *(["-fopenmp"] if parallel else []), "-o", tmp, SRC, "-lm"])
        os.replace(tmp, lib)
    return lib


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("reintroductions", C.c_int),
                ("converged", C.c_int), ("relres", C.c_double), ("rho_avg", C.c_double)]


_libs = {}
COARSENINGS = {"rs": 0, "pmis": 1}


def _load(parallel: bool = False):
    if parallel not in _libs:
        path = LIB_OMP if parallel else LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            build(force=True, parallel=parallel)
        lib = C.CDLL(path)
        P = C.c_void_p
        ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        up = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        lp = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        lib.or_setup.argtypes = [C.c_int, ip, ip, dp, C.c_double, C.c_int, C.c_int, C.c_double,
                                 C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_uint64, C.POINTER(P)]
        lib.or_setup.restype = C.c_int
        lib.or_free.argtypes = [P]
        lib.or_pmis_rounds.argtypes = [C.c_int, ip, ip, dp, ip]
        lib.or_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        lib.or_splitmix64.restype = C.c_uint64
        lib.or_num_levels.argtypes = [P]
        lib.or_num_levels.restype = C.c_int
        lib.or_level_sizes.argtypes = [P, C.c_int, lp]
        lib.or_level_gamma.argtypes = [P, C.c_int]
        lib.or_level_gamma.restype = C.c_double
        lib.or_export.argtypes = [P, C.c_int, C.c_int, ip, ip, dp]
        lib.or_export_mask.argtypes = [P, C.c_int, C.c_int, up]
        lib.or_export_cf.argtypes = [P, C.c_int, ip]
        lib.or_export_rowmax.argtypes = [P, C.c_int, dp]
        lib.or_sparsify.argtypes = [P, dp]
        lib.or_reintroduce.argtypes = [P, C.c_int, C.c_double, C.POINTER(C.c_int)]
        lib.or_set_method.argtypes = [P, C.c_int]
        lib.or_set_relaxation.argtypes = [P, C.c_int, C.c_int]
        lib.or_set_lumping.argtypes = [P, C.c_int]
        lib.or_strong_lump_csr.argtypes = [C.c_int, ip, ip, dp, up, C.c_double, dp]
        lib.or_gs_sweep.argtypes = [C.c_int, ip, ip, dp, dp, dp, dp, C.c_int, C.c_int]
        lib.or_vcycle.argtypes = [P, dp, dp]
        lib.or_level_op.argtypes = [P, C.c_int, C.c_int, dp, dp, dp]
        lib.or_solve.argtypes = [P, dp, dp, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int,
                                 C.c_int, C.c_double, C.c_double, C.POINTER(_Info), P]
        _libs[parallel] = lib
    return _libs[parallel]


@dataclass
class Sparse:
    nrows: int
    ncols: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.nrows, self.ncols))
        rows = np.repeat(np.arange(self.nrows), np.diff(self.row_ptr))
        d[rows, self.col] = self.val
        return d


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


def strong_lump(A, keep, theta: float = 0.25) -> np.ndarray:
    """Values of the kept pattern of the plain matrix A after strong-neighbour
    lumping of the entries whose keep flag is 0."""
    lib = _load()
    keep = np.ascontiguousarray(keep, np.uint8)
    out = np.zeros(max(int(keep.sum()), 1), np.float64)
    rc = lib.or_strong_lump_csr(int(A.n), np.ascontiguousarray(A.row_ptr, np.int32),
                                np.ascontiguousarray(A.col, np.int32), np.ascontiguousarray(A.val, np.float64),
                                keep, float(theta), out)
    if rc != OK:
        raise ValueError(f"strong_lump status {rc}")
    return out[:int(keep.sum())]


def gs_sweep(A, b, x, block: int, forward: bool) -> np.ndarray:
    """One hybrid Gauss-Seidel sweep of the plain matrix A from x."""
    lib = _load()
    out = np.zeros(A.n, np.float64)
    rc = lib.or_gs_sweep(int(A.n), np.ascontiguousarray(A.row_ptr, np.int32), np.ascontiguousarray(A.col, np.int32),
                         np.ascontiguousarray(A.val, np.float64), np.ascontiguousarray(b, np.float64),
                         np.ascontiguousarray(x, np.float64), out, int(block), int(bool(forward)))
    if rc != OK:
        raise ValueError(f"gs_sweep status {rc}")
    return out


class OracleAMG:
    """Oracle hierarchy: Galerkin setup, Sparse Galerkin sparsify, solves."""

    def __init__(self, A, theta=0.25, max_coarse=49, max_levels=25, omega=2.0 / 3.0,
                 nu_pre=1, nu_post=1, nongalerkin_gamma=None, coarsening="rs", seed=0, parallel=False):
        """nongalerkin_gamma: per-level tolerances of the method of non-Galerkin
        coarse grids (each coarse product sparsified during setup); None for the
        Galerkin hierarchy.  coarsening: "rs" (Ruge-Stueben first pass) or
        "pmis" (weights of level l from the SplitMix64 stream seed + l).
        parallel: the OpenMP timing build (the same results, bit for bit)."""
        if coarsening not in COARSENINGS:
            raise ValueError(f"unknown coarsening {coarsening!r}")
        lib = _load(parallel)
        self._lib = lib
        self.n = int(A.n)
        h = C.c_void_p()
        ng = None if nongalerkin_gamma is None else np.ascontiguousarray(nongalerkin_gamma, np.float64)
        rc = lib.or_setup(self.n, np.ascontiguousarray(A.row_ptr, np.int32),
                          np.ascontiguousarray(A.col, np.int32),
                          np.ascontiguousarray(A.val, np.float64),
                          float(theta), int(max_coarse), int(max_levels), float(omega),
                          int(nu_pre), int(nu_post),
                          None if ng is None else ng.ctypes.data_as(C.c_void_p), 0 if ng is None else len(ng),
                          COARSENINGS[coarsening], int(seed) & 0xFFFFFFFFFFFFFFFF, C.byref(h))
        if rc != OK:
            raise ValueError(f"oracle setup failed with status {rc}")
        self._h = h
        self.nlev = lib.or_num_levels(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and self._lib is not None:
            self._lib.or_free(h)
            self._h = None

    def sizes(self, l: int) -> dict:
        out = np.zeros(5, np.int64)
        self._lib.or_level_sizes(self._h, l, out)
        return dict(n=int(out[0]), nnz=int(out[1]), nnz_hat=int(out[2]), nnz_P=int(out[3]),
                    n_coarse=int(out[4]))

    def gamma(self, l: int) -> float:
        return self._lib.or_level_gamma(self._h, l)

    def export(self, l: int, which: str) -> Sparse:
        s = self.sizes(l)
        if which in ("A", "AHAT"):
            nr, nc, nnz = s["n"], s["n"], s["nnz"] if which == "A" else s["nnz_hat"]
        elif which == "P":
            nr, nc, nnz = s["n"], s["n_coarse"], s["nnz_P"]
        elif which == "R":
            nr, nc, nnz = s["n_coarse"], s["n"], s["nnz_P"]
        else:  # S: size unknown up front; bounded by nnz(A)
            nr, nc, nnz = s["n"], s["n"], s["nnz"]
        rp = np.zeros(nr + 1, np.int32)
        ci = np.zeros(max(nnz, 1), np.int32)
        v = np.zeros(max(nnz, 1), np.float64)
        rc = self._lib.or_export(self._h, l, WHICH[which], rp, ci, v)
        if rc != OK:
            raise ValueError(f"export {which} of level {l}: status {rc}")
        m = int(rp[-1])
        return Sparse(nr, nc, rp, ci[:m].copy(), v[:m].copy())

    def mask(self, l: int, which: str) -> np.ndarray:
        out = np.zeros(max(self.sizes(l)["nnz"], 1), np.uint8)
        rc = self._lib.or_export_mask(self._h, l, 0 if which == "M" else 1, out)
        if rc != OK:
            raise ValueError(f"mask {which} of level {l}: status {rc}")
        return out[: self.sizes(l)["nnz"]]

    def cf(self, l: int) -> np.ndarray:
        out = np.zeros(self.sizes(l)["n"], np.int32)
        if self._lib.or_export_cf(self._h, l, out) != OK:
            raise ValueError("no C/F split on the coarsest level")
        return out

    def rowmax(self, l: int) -> np.ndarray:
        out = np.zeros(self.sizes(l)["n"], np.float64)
        self._lib.or_export_rowmax(self._h, l, out)
        return out

    def sparsify(self, gammas) -> None:
        g = np.zeros(self.nlev, np.float64)
        gammas = list(gammas)[: self.nlev]
        g[: len(gammas)] = gammas
        rc = self._lib.or_sparsify(self._h, g)
        if rc != OK:
            raise ValueError(f"sparsify status {rc}")

    def sparsify_from(self, gamma: float, first_level: int = 2) -> None:
        self.sparsify([0.0 if l < first_level else gamma for l in range(self.nlev)])

    def set_method(self, hybrid: bool) -> None:
        """Sparse Galerkin (False) or Hybrid Galerkin (True) for later sparsify /
        reintroduce calls (Section 3, sparse_hybrid_setup)."""
        rc = self._lib.or_set_method(self._h, int(bool(hybrid)))
        if rc != OK:
            raise ValueError(f"set_method status {rc}")

    def set_relaxation(self, kind: str = "jacobi", block: int = 1) -> None:
        """Weighted Jacobi, or hybrid symmetric Gauss-Seidel with blocks of
        `block` rows, for later V-cycles and solves."""
        rc = self._lib.or_set_relaxation(self._h, {"jacobi": 0, "hybrid_gs": 1}[kind], int(block))
        if rc != OK:
            raise ValueError(f"set_relaxation status {rc}")

    def set_lumping(self, mode: str = "diagonal") -> None:
        """Where later sparsify calls put dropped entries: "diagonal"
        (Algorithm 3b) or "strong" (strong neighbours, Algorithm 3)."""
        if mode not in ("diagonal", "strong"):
            raise ValueError(f"unknown lumping {mode!r}")
        rc = self._lib.or_set_lumping(self._h, {"diagonal": 0, "strong": 1}[mode])
        if rc != OK:
            raise ValueError(f"set_lumping status {rc}")

    def reintroduce(self, s: int = 1, gamma_min: float = 0.01):
        first = C.c_int(-1)
        rc = self._lib.or_reintroduce(self._h, int(s), float(gamma_min), C.byref(first))
        return rc, first.value

    def vcycle(self, b: np.ndarray, x: np.ndarray | None = None) -> np.ndarray:
        x = np.zeros(self.n) if x is None else np.array(x, np.float64, copy=True)
        self._lib.or_vcycle(self._h, np.ascontiguousarray(b, np.float64), x)
        return x

    def level_op(self, l: int, op: int, inp: np.ndarray, x: np.ndarray | None, nout: int):
        out = np.zeros(max(nout, 1), np.float64)
        inp = np.ascontiguousarray(inp, np.float64)
        xx = np.ascontiguousarray(x if x is not None else np.zeros(1), np.float64)
        rc = self._lib.or_level_op(self._h, l, op, inp, xx, out)
        if rc != OK:
            raise ValueError(f"level op {op} on level {l}: status {rc}")
        return out[:nout]

    def solve(self, b, x0=None, method=PCG, tol=1e-8, maxit=200, adaptive=False, k=3, s=1,
              rho_max=0.5, gamma_min=0.01):
        x = np.zeros(self.n) if x0 is None else np.array(x0, np.float64, copy=True)
        info = _Info()
        hist = np.full(maxit + 1, np.nan)
        rc = self._lib.or_solve(self._h, np.ascontiguousarray(b, np.float64), x, int(method),
                                float(tol), int(maxit), int(bool(adaptive)), int(k), int(s),
                                float(rho_max), float(gamma_min), C.byref(info),
                                hist.ctypes.data_as(C.c_void_p))
        res = SolveResult(rc, info.iters, info.restarts, info.reintroductions,
                          bool(info.converged), info.relres, info.rho_avg,
                          hist[: info.iters + 1].copy())
        return x, res
