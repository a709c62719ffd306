"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

Holds only input construction (matrix patterns, values, right-hand sides,
instance tables); none of the solver's arithmetic lives here.  The heavy
generators are plain C in ``gen.c`` (compiled with gcc on first use); the
definitions of the counter-based SplitMix64 draws and of the ``stencil7`` /
``randsym`` patterns are stated in that file's header.

The paper benchmarks SuiteSparse matrices (dimension up to 1e6, density below
1%, Table 2 spans 0.6-41 nonzeros per row, Section 6); these generators stand
in for them with the same shapes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libspkgen.so")
_lib = None
_DEV_SRC = os.path.join(_HERE, "gen_device.hip")
_DEV_LIB = os.path.join(_HERE, "libspkgen_dev.so")
_dev_lib = None


def build_device(force: bool = True) -> str:
    """Compile gen_device.hip (hipcc, gfx950, no FP contraction) into libspkgen_dev.so."""
    if force or not os.path.exists(_DEV_LIB):
        tmp = _DEV_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-fPIC", "-shared",
                               "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               _DEV_SRC, "-o", tmp])
        os.replace(tmp, _DEV_LIB)
    return _DEV_LIB


def _get_dev():
    global _dev_lib
    if _dev_lib is None:
        if not os.path.exists(_DEV_LIB):
            build_device()
        lib = ctypes.CDLL(_DEV_LIB)
        vp = ctypes.c_void_p
        lib.gen_dev_stencil7.restype = ctypes.c_int
        lib.gen_dev_stencil7.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int, vp, vp, vp,
                                         ctypes.c_int, vp]
        lib.gen_dev_vec.restype = ctypes.c_int
        lib.gen_dev_vec.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, vp, vp]
        _dev_lib = lib
    return _dev_lib


def dev_stencil7(N: int, seed: int, delta: float = 1.0, f32x: bool = False, val_f32: bool = False,
                 device: str = "cuda:0"):
    """stencil7(N) generated on the GPU: (row_ptr int64, col int32, val f64/f32) torch tensors,
    bit-identical to stencil7(N, seed, delta, f32x) from the host generator."""
    import torch
    n = N ** 3
    nnz = stencil7_nnz(N)
    rp = torch.empty(n + 1, dtype=torch.int64, device=device)
    col = torch.empty(nnz, dtype=torch.int32, device=device)
    val = torch.empty(nnz, dtype=torch.float32 if val_f32 else torch.float64, device=device)
    stream = torch.cuda.current_stream(device).cuda_stream
    rc = _get_dev().gen_dev_stencil7(N, seed, float(delta), int(f32x), rp.data_ptr(), col.data_ptr(),
                                     val.data_ptr(), int(val_f32), stream)
    if rc != 0:
        raise RuntimeError("gen_dev_stencil7 failed (hipError %d)" % rc)
    return rp, col, val


def dev_vec(n: int, seed: int, stream_id: int, device: str = "cuda:0"):
    """Uniform[-1,1) vector on the GPU; dev_vec(n, seed, 2) equals rhs(n, seed)."""
    import torch
    b = torch.empty(n, dtype=torch.float64, device=device)
    rc = _get_dev().gen_dev_vec(n, seed, stream_id, b.data_ptr(), torch.cuda.current_stream(device).cuda_stream)
    if rc != 0:
        raise RuntimeError("gen_dev_vec failed (hipError %d)" % rc)
    return b


def build(force: bool = False) -> str:
    """Compile gen.c into libspkgen.so (gcc, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, u64, f64, i32, vp = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_void_p)
        lib.gen_hash.restype = u64
        lib.gen_hash.argtypes = [u64, u64, u64]
        lib.gen_unif_f64.restype = f64
        lib.gen_unif_f64.argtypes = [u64, u64, u64]
        lib.gen_unif_f32x.restype = f64
        lib.gen_unif_f32x.argtypes = [u64, u64, u64]
        lib.gen_stencil7_nnz.restype = i64
        lib.gen_stencil7_nnz.argtypes = [i64]
        lib.gen_stencil7.restype = i32
        lib.gen_stencil7.argtypes = [i64, u64, f64, i32, vp, vp, vp]
        lib.gen_randsym_max_nnz.restype = i64
        lib.gen_stencil7_ns.restype = i32
        lib.gen_stencil7_ns.argtypes = [i64, u64, f64, vp, vp, vp]
        lib.gen_randsym_max_nnz.argtypes = [i64, i32]
        lib.gen_randsym.restype = i64
        lib.gen_randsym.argtypes = [i64, u64, f64, i32, i32, vp, vp, vp]
        lib.gen_stencil7_row.restype = i32
        lib.gen_stencil7_row.argtypes = [i64, u64, f64, i32, i64, vp, vp]
        lib.gen_stencil7_block.restype = i64
        lib.gen_stencil7_block.argtypes = [i64, u64, f64, i32, i64, i64, vp, vp, vp]
        lib.gen_rhs.restype = None
        lib.gen_rhs.argtypes = [i64, u64, vp]
        lib.gen_vec.restype = None
        lib.gen_vec.argtypes = [i64, u64, u64, vp]
        lib.gen_instances.restype = None
        lib.gen_instances.argtypes = [i64, u64, f64, f64, vp, vp]
        lib.gen_powerlaw_max_nnz.restype = i64
        lib.gen_powerlaw_max_nnz.argtypes = [i64, i32, i64, i64]
        lib.gen_powerlaw.restype = i64
        lib.gen_powerlaw.argtypes = [i64, u64, f64, i32, i64, i64, i64, i32, vp, vp, vp]
        lib.gen_powerlaw_hub.restype = None
        lib.gen_powerlaw_hub.argtypes = [i64, u64, i64, i64, i64, vp, vp]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class CSR:
    """Host CSR matrix: row_ptr int64[n+1], col int32/int64[nnz], val float64[nnz]."""
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1]) if self.row_ptr.size else 0

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n_rows, self.n_cols))
        for i in range(self.n_rows):
            for k in range(int(self.row_ptr[i]), int(self.row_ptr[i + 1])):
                a[i, int(self.col[k])] += self.val[k]
        return a


# ---------------------------------------------------------------- draws
def hash64(seed: int, stream: int, ctr: int) -> int:
    return int(_get().gen_hash(seed, stream, ctr))


def unif(seed: int, stream: int, ctr: int) -> float:
    return float(_get().gen_unif_f64(seed, stream, ctr))


def unif_f32x(seed: int, stream: int, ctr: int) -> float:
    return float(_get().gen_unif_f32x(seed, stream, ctr))


# ---------------------------------------------------------------- matrices
def stencil7_nnz(N: int) -> int:
    return int(_get().gen_stencil7_nnz(N))


def stencil7(N: int, seed: int, delta: float = 1.0, f32x: bool = False) -> CSR:
    n = N * N * N
    nnz = stencil7_nnz(N)
    rp = np.empty(n + 1, np.int64)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    rc = _get().gen_stencil7(N, seed, float(delta), int(f32x), _p(rp), _p(col), _p(val))
    if rc != 0:
        raise ValueError("stencil7: N must be >= 1")
    return CSR(n, n, rp, col, val)


def stencil7_ns(N: int, seed: int, delta: float = 1.0) -> CSR:
    """Nonsymmetric stencil7: independent draws for a_ij and a_ji (stream 16),
    strictly row diagonally dominant."""
    n = N * N * N
    nnz = stencil7_nnz(N)
    rp = np.empty(n + 1, np.int64)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    if _get().gen_stencil7_ns(N, seed, float(delta), _p(rp), _p(col), _p(val)) != 0:
        raise ValueError("stencil7_ns: N must be >= 1")
    return CSR(n, n, rp, col, val)


def randsym(n: int, seed: int, delta: float = 1.0, deg: int = 3, f32x: bool = False) -> CSR:
    cap = int(_get().gen_randsym_max_nnz(n, deg))
    rp = np.empty(n + 1, np.int64)
    col = np.empty(cap, np.int32)
    val = np.empty(cap, np.float64)
    nnz = int(_get().gen_randsym(n, seed, float(delta), deg, int(f32x), _p(rp), _p(col), _p(val)))
    if nnz < 0:
        raise ValueError("randsym: bad arguments or out of memory (%d)" % nnz)
    return CSR(n, n, rp, col[:nnz].copy(), val[:nnz].copy())


def powerlaw(n: int, seed: int, hubs: int = 16, lo: int = 1000, hi: int = 10000, delta: float = 1.0,
             deg: int = 3, f32x: bool = False) -> CSR:
    """randsym(n) plus `hubs` hub rows of lo..hi partners (log-uniform): a
    heavy-tailed row-length mix (symmetric, diagonally dominant, SPD)."""
    cap = int(_get().gen_powerlaw_max_nnz(n, deg, hubs, hi))
    rp = np.empty(n + 1, np.int64)
    col = np.empty(cap, np.int32)
    val = np.empty(cap, np.float64)
    nnz = int(_get().gen_powerlaw(n, seed, float(delta), deg, hubs, lo, hi, int(f32x), _p(rp), _p(col), _p(val)))
    if nnz < 0:
        raise ValueError("powerlaw: bad arguments or out of memory (%d)" % nnz)
    return CSR(n, n, rp, col[:nnz].copy(), val[:nnz].copy())


def powerlaw_hubs(n: int, seed: int, hubs: int = 16, lo: int = 1000, hi: int = 10000):
    """(row, partner draws) of every hub of powerlaw(n, seed, hubs, lo, hi)."""
    out = []
    r = ctypes.c_int64()
    d = ctypes.c_int64()
    for h in range(hubs):
        _get().gen_powerlaw_hub(n, seed, h, lo, hi, ctypes.byref(r), ctypes.byref(d))
        out.append((r.value, d.value))
    return out


def randsym_many(specs, threads: int = 0):
    """randsym(n, seed) for every (n, seed) in specs, built on several host
    threads (each build is one C call); returns the CSR list in order."""
    from concurrent.futures import ThreadPoolExecutor
    workers = threads if threads > 0 else min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda sp: randsym(int(sp[0]), int(sp[1])), specs))


def serving_mix(count: int = 256, seed: int = 4, lo: float = 1e3, hi: float = 1e6, threads: int = 0):
    """The serving workload: count randsym instances with log-uniform sizes in
    [lo, hi] and per-instance seeds; returns (matrices, right-hand sides)."""
    sizes, seeds = instances(count, seed, lo, hi)
    specs = [(int(n), int(sd) % (1 << 31)) for n, sd in zip(sizes, seeds)]
    mats = randsym_many(specs, threads)
    return mats, [rhs(n, sd) for n, sd in specs]


def stencil7_rows(N: int, seed: int, rows, delta: float = 1.0, f32x: bool = False):
    """Entries of selected rows of stencil7(N) without building the matrix:
    list of (cols int64 array, vals float64 array), from the host generator."""
    out = []
    cols = np.empty(7, np.int64)
    vals = np.empty(7, np.float64)
    for i in rows:
        m = int(_get().gen_stencil7_row(N, seed, float(delta), int(f32x), int(i), _p(cols), _p(vals)))
        out.append((cols[:m].copy(), vals[:m].copy()))
    return out


def stencil7_block(N: int, seed: int, r0: int, r1: int, delta: float = 1.0, f32x: bool = False):
    """Rows [r0, r1) of stencil7(N) without building the matrix: (row_ptr
    int64 starting at 0, global column indices int64, values float64)."""
    m = r1 - r0
    rp = np.empty(m + 1, np.int64)
    col = np.empty(7 * max(m, 0), np.int64)
    val = np.empty(7 * max(m, 0), np.float64)
    k = int(_get().gen_stencil7_block(N, seed, float(delta), int(f32x), r0, r1, _p(rp), _p(col), _p(val)))
    if k < 0:
        raise ValueError("stencil7_block: bad row range")
    return rp, col[:k], val[:k]


def rhs(n: int, seed: int) -> np.ndarray:
    b = np.empty(n, np.float64)
    _get().gen_rhs(n, seed, _p(b))
    return b


def vec(n: int, seed: int, stream: int) -> np.ndarray:
    v = np.empty(n, np.float64)
    _get().gen_vec(n, seed, stream, _p(v))
    return v


def instances(count: int, seed: int, lo: float = 1e3, hi: float = 1e6):
    """Serving workload: sizes log-uniform in [lo, hi] and per-instance seeds."""
    sizes = np.empty(count, np.int64)
    seeds = np.empty(count, np.uint64)
    _get().gen_instances(count, seed, float(lo), float(hi), _p(sizes), _p(seeds))
    return sizes, seeds


# ---------------------------------------------------------------- small structured inputs
def from_dense(a: np.ndarray, keep_zeros: bool = False) -> CSR:
    a = np.asarray(a, dtype=np.float64)
    n_rows, n_cols = a.shape
    rp = [0]
    cols, vals = [], []
    for i in range(n_rows):
        for j in range(n_cols):
            if keep_zeros or a[i, j] != 0.0:
                cols.append(j)
                vals.append(a[i, j])
        rp.append(len(cols))
    return CSR(n_rows, n_cols, np.array(rp, np.int64), np.array(cols, np.int32),
               np.array(vals, np.float64))


def diagonal(d) -> CSR:
    d = np.asarray(d, np.float64)
    n = d.size
    return CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), d.copy())


def laplacian1d(n: int) -> CSR:
    """tridiag(-1, 2, -1) of size n."""
    rp = [0]
    cols, vals = [], []
    for i in range(n):
        if i > 0:
            cols.append(i - 1); vals.append(-1.0)
        cols.append(i); vals.append(2.0)
        if i < n - 1:
            cols.append(i + 1); vals.append(-1.0)
        rp.append(len(cols))
    return CSR(n, n, np.array(rp, np.int64), np.array(cols, np.int32), np.array(vals, np.float64))


def permutation(n: int, seed: int) -> CSR:
    """Permutation matrix; the permutation is an argsort of seeded draws."""
    keys = np.array([hash64(seed, 7, i) for i in range(n)], dtype=np.uint64)
    perm = np.argsort(keys, kind="stable")
    return CSR(n, n, np.arange(n + 1, dtype=np.int64), perm.astype(np.int32), np.ones(n))


def dyadic_random(n_rows: int, n_cols: int, per_row: int, seed: int) -> CSR:
    """Values in {-1,-1/2,1/2,1}: every partial sum with small-integer x is exact."""
    choices = np.array([-1.0, -0.5, 0.5, 1.0])
    rp = [0]
    cols, vals = [], []
    for i in range(n_rows):
        picked = set()
        for t in range(per_row):
            j = hash64(seed, 8, i * per_row + t) % n_cols
            if j in picked:
                continue
            picked.add(j)
        for j in sorted(picked):
            cols.append(j)
            vals.append(choices[hash64(seed, 9, i * n_cols + j) % 4])
        rp.append(len(cols))
    return CSR(n_rows, n_cols, np.array(rp, np.int64), np.array(cols, np.int32),
               np.array(vals, np.float64))
