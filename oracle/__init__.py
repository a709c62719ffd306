"""FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product library never loads it, and it
shares no code with the HIP path.

The arithmetic lives in ``oracle.c`` (plain C, FP64, single thread, no FP
contraction); this module only marshals numpy arrays.  Every function states
the definition it follows in ``oracle.c``: the CSR SpMV definition (the
operator apply of Section 4.2 / the SpMV benchmark of Section 6.1), textbook
Hestenes-Stiefel CG (the CG solver benchmarked in Section 6.2) with the
Iteration / ResidualNorm(rhs_norm) criteria of the Section 3.5 configuration
example, CGS (the other Krylov solver of Section 6.2, Barrett et al.
template), CG with the scalar Jacobi preconditioner of the Section 3.5
example (Saad Alg. 9.1), restarted GMRES(m) with modified Gram-Schmidt and
Givens rotations (the solver of the Section 3.5 listings; Saad Alg. 6.9),
the nnz-balanced row partition and the Gershgorin condition bound.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# Stop reasons and CSR verdicts, as numbered in oracle.c.
RUNNING, CONVERGED, MAX_ITERS, BREAKDOWN, NON_FINITE = 0, 1, 2, 3, 4
CSR_OK, CSR_BAD_SIZE, CSR_BAD_FIRST, CSR_DECREASING, CSR_BAD_LAST, CSR_BAD_COLUMN = range(6)

CFLAGS = ["-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = False, src: str = _SRC, out: str = _LIB, extra=()) -> str:
    """Compile oracle.c with gcc.  ``src``/``out``/``extra`` let tests build variants."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, *extra, src, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


class CGResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("stop_reason", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("rhs_norm", ctypes.c_double),
                ("implicit_resnorm", ctypes.c_double), ("true_resnorm", ctypes.c_double)]


def load(path: str = _LIB):
    vp, i64, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    lib = ctypes.CDLL(path)
    lib.orc_csr_validate.restype = ctypes.c_int
    lib.orc_csr_validate.argtypes = [i64, i64, i64, vp, vp]
    lib.orc_spmv.restype = None
    lib.orc_spmv.argtypes = [i64, vp, vp, vp, vp, vp]
    lib.orc_spmv_abs.restype = None
    lib.orc_spmv_abs.argtypes = [i64, vp, vp, vp, vp, vp]
    lib.orc_residual.restype = None
    lib.orc_residual.argtypes = [i64, vp, vp, vp, vp, vp, vp]
    lib.orc_residual_sumsq.restype = f64
    lib.orc_residual_sumsq.argtypes = [i64, vp, vp, vp, vp, vp]
    lib.orc_cg.restype = ctypes.c_int
    lib.orc_cg.argtypes = [i64, vp, vp, vp, vp, vp, f64, i64, ctypes.POINTER(CGResult), vp]
    lib.orc_cgs.restype = ctypes.c_int
    lib.orc_cgs.argtypes = [i64, vp, vp, vp, vp, vp, f64, i64, ctypes.POINTER(CGResult), vp]
    lib.orc_pcg_jacobi.restype = ctypes.c_int
    lib.orc_pcg_jacobi.argtypes = [i64, vp, vp, vp, vp, vp, f64, i64, ctypes.POINTER(CGResult), vp]
    lib.orc_gmres.restype = ctypes.c_int
    lib.orc_gmres.argtypes = [i64, vp, vp, vp, vp, vp, f64, i64, i64, ctypes.POINTER(CGResult), vp]
    lib.orc_cgs_jacobi.restype = ctypes.c_int
    lib.orc_cgs_jacobi.argtypes = [i64, vp, vp, vp, vp, vp, f64, i64, ctypes.POINTER(CGResult), vp]
    lib.orc_gmres_jacobi.restype = ctypes.c_int
    lib.orc_gmres_jacobi.argtypes = [i64, vp, vp, vp, vp, vp, f64, i64, i64, ctypes.POINTER(CGResult), vp]
    lib.orc_diagonal.restype = None
    lib.orc_diagonal.argtypes = [i64, vp, vp, vp, vp]
    lib.orc_coo_spmv.restype = None
    lib.orc_coo_spmv.argtypes = [i64, i64, vp, vp, vp, vp, vp]
    lib.orc_coo_validate.restype = ctypes.c_int
    lib.orc_coo_validate.argtypes = [i64, i64, i64, vp, vp, ctypes.POINTER(ctypes.c_int)]
    lib.orc_partition.restype = None
    lib.orc_partition.argtypes = [i64, vp, i64, vp]
    lib.orc_gershgorin_kappa.restype = f64
    lib.orc_gershgorin_kappa.argtypes = [i64, vp, vp, vp]
    return lib


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = load(_LIB)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr64(A):
    return (np.ascontiguousarray(A.row_ptr, np.int64), np.ascontiguousarray(A.col, np.int64),
            np.ascontiguousarray(A.val, np.float64))


class Oracle:
    """Bound oracle functions; ``lib`` may be a variant build (tests plant mistakes there)."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else _get()

    def csr_validate(self, n_rows, n_cols, nnz, row_ptr, col) -> int:
        rp = np.ascontiguousarray(row_ptr, np.int64)
        ci = np.ascontiguousarray(col, np.int64)
        if rp.size < max(n_rows, 0) + 1:
            raise ValueError("row_ptr must hold n_rows + 1 entries")
        return int(self.lib.orc_csr_validate(n_rows, n_cols, nnz, _p(rp), _p(ci)))

    def spmv(self, A, x) -> np.ndarray:
        rp, ci, va = _csr64(A)
        x = np.ascontiguousarray(x, np.float64)
        y = np.empty(A.n_rows, np.float64)
        self.lib.orc_spmv(A.n_rows, _p(rp), _p(ci), _p(va), _p(x), _p(y))
        return y

    def coo_spmv(self, n_rows, row, col, val, x) -> np.ndarray:
        """COO product from its definition (entries in any order, duplicates summed)."""
        row = np.ascontiguousarray(row, np.int64)
        col = np.ascontiguousarray(col, np.int64)
        val = np.ascontiguousarray(val, np.float64)
        x = np.ascontiguousarray(x, np.float64)
        y = np.empty(n_rows, np.float64)
        self.lib.orc_coo_spmv(n_rows, row.size, _p(row), _p(col), _p(val), _p(x), _p(y))
        return y

    def coo_validate(self, n_rows, n_cols, row, col):
        """(verdict, row_sorted) of a COO matrix."""
        row = np.ascontiguousarray(row, np.int64)
        col = np.ascontiguousarray(col, np.int64)
        srt = ctypes.c_int(0)
        v = self.lib.orc_coo_validate(n_rows, n_cols, row.size, _p(row), _p(col), ctypes.byref(srt))
        return int(v), bool(srt.value)

    def spmv_abs(self, A, x) -> np.ndarray:
        rp, ci, va = _csr64(A)
        x = np.ascontiguousarray(x, np.float64)
        y = np.empty(A.n_rows, np.float64)
        self.lib.orc_spmv_abs(A.n_rows, _p(rp), _p(ci), _p(va), _p(x), _p(y))
        return y

    def residual(self, A, b, x) -> np.ndarray:
        rp, ci, va = _csr64(A)
        b = np.ascontiguousarray(b, np.float64)
        x = np.ascontiguousarray(x, np.float64)
        r = np.empty(A.n_rows, np.float64)
        self.lib.orc_residual(A.n_rows, _p(rp), _p(ci), _p(va), _p(b), _p(x), _p(r))
        return r

    def residual_norm_rows(self, blocks, make_block, b, x, threads: int = 1) -> float:
        """||b - A x||_2 for a matrix visited block by block (never held whole).

        blocks: (r0, r1) row ranges covering the matrix's rows once;
        make_block(r0, r1) returns those rows as (row_ptr from 0, global column
        indices, values).  Each block's squared residual is summed by
        orc_residual_sumsq; the block totals are added in the order of
        ``blocks`` (threads only overlap the block builds and sums), then the
        square root is taken."""
        b = np.ascontiguousarray(b, np.float64)
        x = np.ascontiguousarray(x, np.float64)

        def one(rng):
            r0, r1 = rng
            rp, ci, va = make_block(r0, r1)
            rp = np.ascontiguousarray(rp, np.int64)
            ci = np.ascontiguousarray(ci, np.int64)
            va = np.ascontiguousarray(va, np.float64)
            bb = b[r0:r1]
            return float(self.lib.orc_residual_sumsq(r1 - r0, _p(rp), _p(ci), _p(va), _p(bb), _p(x)))

        blocks = list(blocks)
        if threads > 1:
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(max_workers=threads) as ex:
                parts = list(ex.map(one, blocks))
        else:
            parts = [one(r) for r in blocks]
        total = 0.0
        for v in parts:
            total += v
        return math.sqrt(total)

    def _krylov(self, fn, A, b, x0, tau, max_iters, history):
        rp, ci, va = _csr64(A)
        n = A.n_rows
        b = np.ascontiguousarray(b, np.float64)
        x = np.zeros(n) if x0 is None else np.array(x0, np.float64, copy=True)
        res = CGResult()
        hist = np.full(max_iters + 1, np.nan) if history else None
        fn(n, _p(rp), _p(ci), _p(va), _p(b), _p(x), float(tau), int(max_iters), ctypes.byref(res), _p(hist))
        if hist is not None:
            hist = hist[: res.iterations + 1]
        return x, res, hist

    def cg(self, A, b, x0=None, tau=1e-14, max_iters=10000, history=False):
        """Textbook CG.  Returns (x, CGResult, hist or None)."""
        return self._krylov(self.lib.orc_cg, A, b, x0, tau, max_iters, history)

    def cgs(self, A, b, x0=None, tau=1e-14, max_iters=10000, history=False):
        """CGS (Barrett et al. template, shadow residual r0).  Returns (x, CGResult, hist or None)."""
        return self._krylov(self.lib.orc_cgs, A, b, x0, tau, max_iters, history)

    def pcg_jacobi(self, A, b, x0=None, tau=1e-14, max_iters=10000, history=False):
        """CG preconditioned by diag(A).  Returns (x, CGResult, hist or None)."""
        return self._krylov(self.lib.orc_pcg_jacobi, A, b, x0, tau, max_iters, history)

    def gmres(self, A, b, x0=None, tau=1e-14, max_iters=10000, m=30, history=False, jacobi=False):
        """Restarted GMRES(m), MGS Arnoldi, Givens rotations; jacobi: M = diag(A) on the right.
        Returns (x, CGResult, hist or None)."""
        rp, ci, va = _csr64(A)
        n = A.n_rows
        b = np.ascontiguousarray(b, np.float64)
        x = np.zeros(n) if x0 is None else np.array(x0, np.float64, copy=True)
        res = CGResult()
        hist = np.full(max_iters + 1, np.nan) if history else None
        fn = self.lib.orc_gmres_jacobi if jacobi else self.lib.orc_gmres
        fn(n, _p(rp), _p(ci), _p(va), _p(b), _p(x), float(tau), int(max_iters), int(m), ctypes.byref(res), _p(hist))
        if hist is not None:
            hist = hist[: res.iterations + 1]
        return x, res, hist

    def cgs_jacobi(self, A, b, x0=None, tau=1e-14, max_iters=10000, history=False):
        """CGS with M = diag(A) on the right.  Returns (x, CGResult, hist or None)."""
        return self._krylov(self.lib.orc_cgs_jacobi, A, b, x0, tau, max_iters, history)

    def diagonal(self, A) -> np.ndarray:
        rp, ci, va = _csr64(A)
        d = np.empty(A.n_rows, np.float64)
        self.lib.orc_diagonal(A.n_rows, _p(rp), _p(ci), _p(va), _p(d))
        return d

    def partition(self, row_ptr, parts: int) -> np.ndarray:
        rp = np.ascontiguousarray(row_ptr, np.int64)
        split = np.empty(parts + 1, np.int64)
        self.lib.orc_partition(rp.size - 1, _p(rp), parts, _p(split))
        return split

    def gershgorin_kappa(self, A) -> float:
        rp, ci, va = _csr64(A)
        return float(self.lib.orc_gershgorin_kappa(A.n_rows, _p(rp), _p(ci), _p(va)))


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def spmv(A, x):
    return default().spmv(A, x)


def spmv_abs(A, x):
    return default().spmv_abs(A, x)


def coo_spmv(n_rows, row, col, val, x):
    return default().coo_spmv(n_rows, row, col, val, x)


def coo_validate(n_rows, n_cols, row, col):
    return default().coo_validate(n_rows, n_cols, row, col)


def residual(A, b, x):
    return default().residual(A, b, x)


def residual_norm_rows(blocks, make_block, b, x, threads=1):
    return default().residual_norm_rows(blocks, make_block, b, x, threads)


def cg_many(systems, tau=1e-14, max_iters=10000, threads=0):
    """oracle CG on independent systems [(A, b), ...], several at once on host
    threads (each solve is the single-threaded cg above); list of (x, result)."""
    from concurrent.futures import ThreadPoolExecutor
    workers = threads if threads > 0 else min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda s: cg(s[0], s[1], tau=tau, max_iters=max_iters)[:2], systems))


def cg(A, b, x0=None, tau=1e-14, max_iters=10000, history=False):
    return default().cg(A, b, x0, tau, max_iters, history)


def cgs(A, b, x0=None, tau=1e-14, max_iters=10000, history=False):
    return default().cgs(A, b, x0, tau, max_iters, history)


def pcg_jacobi(A, b, x0=None, tau=1e-14, max_iters=10000, history=False):
    return default().pcg_jacobi(A, b, x0, tau, max_iters, history)


def diagonal(A):
    return default().diagonal(A)


def gmres(A, b, x0=None, tau=1e-14, max_iters=10000, m=30, history=False, jacobi=False):
    return default().gmres(A, b, x0, tau, max_iters, m, history, jacobi)


def cgs_jacobi(A, b, x0=None, tau=1e-14, max_iters=10000, history=False):
    return default().cgs_jacobi(A, b, x0, tau, max_iters, history)


def csr_validate(n_rows, n_cols, nnz, row_ptr, col):
    return default().csr_validate(n_rows, n_cols, nnz, row_ptr, col)


def partition(row_ptr, parts):
    return default().partition(row_ptr, parts)


def gershgorin_kappa(A):
    return default().gershgorin_kappa(A)
