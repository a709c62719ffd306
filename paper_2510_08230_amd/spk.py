"""Python binding of the spk C ABI (include/spk.h).

Argument marshalling only: every step of the hot path runs in libspk.so's
HIP kernels.  Functions carry the C names; tensors are torch tensors on a
HIP device (their data_ptr() is passed through, zero-copy), and a non-OK
status raises SpkError with the library's message.  There is no CPU
fallback: if libspk.so is missing or fails to load, importing this module
raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libspk.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libspk.so is not built; run __graft_entry__.build() (hipcc, gfx950) first")
_lib = ctypes.CDLL(LIB_PATH)

# ---- enums (values as in include/spk.h)
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_OUT_OF_MEMORY, ERR_BUDGET, ERR_DEVICE, ERR_INTERNAL = range(7)
F64, F32, F16, BF16 = range(4)
I32, I64 = range(2)
CSR_OK, CSR_BAD_SIZE, CSR_BAD_FIRST, CSR_DECREASING, CSR_BAD_LAST, CSR_BAD_COLUMN = range(6)
STOP_RUNNING, STOP_CONVERGED, STOP_MAX_ITERS, STOP_BREAKDOWN, STOP_NON_FINITE = range(5)
SOLVER_CG, SOLVER_CGS, SOLVER_GMRES = 0, 1, 2
PRECOND_NONE, PRECOND_JACOBI = 0, 1
PREC_FP64, PREC_MIXED_FP32, PREC_MIXED_BF16, PREC_MIXED_FP16 = range(4)
EXEC_AUTO, EXEC_HOST_LOOP, EXEC_GRAPH, EXEC_PERSISTENT = range(4)


class SpkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (spk_status_string(status), msg))
        self.status = status


class Csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("ptr_type", ctypes.c_int32), ("idx_type", ctypes.c_int32), ("val_type", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("values", ctypes.c_void_p)]


class Coo(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("idx_type", ctypes.c_int32), ("val_type", ctypes.c_int32), ("row_idx", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("values", ctypes.c_void_p)]


class SolverCfg(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int32), ("precision", ctypes.c_int32), ("baseline", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("max_iters", ctypes.c_int64), ("reduction_factor", ctypes.c_double),
                ("exec_mode", ctypes.c_int32), ("chunk_iters", ctypes.c_int32), ("record_history", ctypes.c_int32),
                ("true_residual", ctypes.c_int32), ("inner_reduction", ctypes.c_double),
                ("max_outer", ctypes.c_int64), ("krylov_dim", ctypes.c_int64), ("reserved", ctypes.c_int64 * 3)]


class Log(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("outer_iterations", ctypes.c_int64),
                ("implicit_resnorm", ctypes.c_double), ("true_resnorm", ctypes.c_double),
                ("rhs_norm", ctypes.c_double), ("converged", ctypes.c_int32), ("stop_reason", ctypes.c_int32),
                ("elapsed_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PlanInfo(ctypes.Structure):
    _fields_ = [("spmv_kernel", ctypes.c_int32), ("lanes", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("exec_mode", ctypes.c_int32), ("chunk_iters", ctypes.c_int32),
                ("tuned", ctypes.c_int32), ("col_codes", ctypes.c_int32), ("spmv_ms", ctypes.c_double),
                ("fused_loop", ctypes.c_int32), ("nontemporal", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("ticks", ctypes.c_int64), ("peak_slots", ctypes.c_int64),
                ("peak_bytes", ctypes.c_int64), ("budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int64),
                ("peak_device_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp, _i32, _i64, _f64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_P = ctypes.POINTER
_SIGS = {
    "spk_solver_cfg_default": (None, [_P(SolverCfg)]),
    "spk_init": (ctypes.c_int, [ctypes.c_int, _vp, _P(_vp)]),
    "spk_finalize": (ctypes.c_int, [_vp]),
    "spk_last_error": (ctypes.c_char_p, [_vp]),
    "spk_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "spk_csr_check": (ctypes.c_int, [_vp, _P(Csr), _P(_i32)]),
    "spk_partition": (ctypes.c_int, [_vp, _P(Csr), _i64, _vp]),
    "spk_plan_spmv": (ctypes.c_int, [_vp, _P(Csr), _P(_vp)]),
    "spk_coo_check": (ctypes.c_int, [_vp, _P(Coo), _P(_i32), _P(_i32)]),
    "spk_plan_spmv_coo": (ctypes.c_int, [_vp, _P(Coo), _P(_vp)]),
    "spk_plan_solve": (ctypes.c_int, [_vp, _P(Csr), _P(SolverCfg), _P(_vp)]),
    "spk_execute_spmv": (ctypes.c_int, [_vp, _vp, _vp]),
    "spk_execute_solve": (ctypes.c_int, [_vp, _vp, _vp, _P(Log)]),
    "spk_plan_history": (ctypes.c_int, [_vp, _vp, _i64, _P(_i64)]),
    "spk_plan_get_info": (ctypes.c_int, [_vp, _P(PlanInfo)]),
    "spk_plan_set_profiling": (ctypes.c_int, [_vp, _i32]),
    "spk_plan_kernel_stats": (ctypes.c_int, [_vp, _P(_f64), _P(_i64)]),
    "spk_free": (ctypes.c_int, [_vp]),
    "spk_stream_copy": (ctypes.c_int, [_vp, _vp, _vp, _sz, _P(_f64)]),
    "spk_gather_probe": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _vp, _P(_f64)]),
    "spk_solve_noalloc": (ctypes.c_int, [_vp, _P(Csr), _P(SolverCfg), _vp, _vp, _P(Log)]),
    "spk_noalloc_max_rows": (_i64, []),
    "spk_server_request_bytes": (_sz, [_i64, _i64]),
    "spk_server_request_bytes_prec": (_sz, [_i32, _i64, _i64]),
    "spk_server_request_bytes_csr": (_sz, [_P(Csr), _i32]),
    "spk_server_create": (ctypes.c_int, [_vp, _sz, _i32, _P(SolverCfg), _P(_vp)]),
    "spk_server_submit": (ctypes.c_int, [_vp, _P(Csr), _vp, _vp, _P(ctypes.c_uint64)]),
    "spk_server_submit_cfg": (ctypes.c_int, [_vp, _P(Csr), _vp, _vp, _P(SolverCfg), _P(ctypes.c_uint64)]),
    "spk_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, _P(_i32), _P(Log), _P(_i64)]),
    "spk_server_drain": (ctypes.c_int, [_vp]),
    "spk_server_get_stats": (ctypes.c_int, [_vp, _P(ServerStats)]),
    "spk_server_last_error": (ctypes.c_char_p, [_vp]),
    "spk_server_destroy": (ctypes.c_int, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = sorted(_SIGS)


def spk_status_string(status: int) -> str:
    return _lib.spk_status_string(status).decode()


def spk_last_error(ctx) -> str:
    return _lib.spk_last_error(ctx.handle if isinstance(ctx, Context) else ctx).decode()


def _check(status, ctx):
    if status != OK:
        raise SpkError(status, spk_last_error(ctx) if ctx is not None else "")


def _dev_ptr(t, what):
    if t is None:
        return None
    if not getattr(t, "is_cuda", False):
        raise ValueError("%s must be a tensor on a HIP device" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    return ctypes.c_void_p(t.data_ptr())


_TORCH_VAL = {"torch.float64": F64, "torch.float32": F32, "torch.float16": F16, "torch.bfloat16": BF16}
_TORCH_IDX = {"torch.int32": I32, "torch.int64": I64}


class Context:
    def __init__(self, handle):
        self.handle = handle


class CsrMatrix:
    """Device CSR descriptor; keeps the borrowed tensors alive."""

    def __init__(self, row_ptr, col_idx, values, n_rows, n_cols):
        self.tensors = (row_ptr, col_idx, values)
        if row_ptr.dim() != 1 or col_idx.dim() != 1 or values.dim() != 1:
            raise ValueError("CSR arrays must be 1-D")
        if row_ptr.numel() != int(n_rows) + 1 or values.numel() != col_idx.numel():
            raise ValueError("row_ptr must hold n_rows + 1 entries and values as many as col_idx")
        self.desc = Csr()
        self.desc.n_rows = int(n_rows)
        self.desc.n_cols = int(n_cols)
        self.desc.nnz = int(col_idx.numel()) if col_idx is not None else 0
        self.desc.ptr_type = _TORCH_IDX[str(row_ptr.dtype)]
        self.desc.idx_type = _TORCH_IDX[str(col_idx.dtype)]
        self.desc.val_type = _TORCH_VAL[str(values.dtype)]
        self.desc.row_ptr = _dev_ptr(row_ptr, "row_ptr") if row_ptr.numel() else None
        self.desc.col_idx = _dev_ptr(col_idx, "col_idx") if col_idx.numel() else None
        self.desc.values = _dev_ptr(values, "values") if values.numel() else None


class CooMatrix:
    """Device COO descriptor (entries sorted by row); keeps the borrowed tensors alive."""

    def __init__(self, row_idx, col_idx, values, n_rows, n_cols):
        self.tensors = (row_idx, col_idx, values)
        if row_idx.dim() != 1 or col_idx.dim() != 1 or values.dim() != 1:
            raise ValueError("COO arrays must be 1-D")
        if not (row_idx.numel() == col_idx.numel() == values.numel()):
            raise ValueError("row_idx, col_idx and values must have nnz entries each")
        if row_idx.dtype != col_idx.dtype:
            raise ValueError("row_idx and col_idx must share one index type")
        self.desc = Coo()
        self.desc.n_rows = int(n_rows)
        self.desc.n_cols = int(n_cols)
        self.desc.nnz = int(values.numel())
        self.desc.idx_type = _TORCH_IDX[str(col_idx.dtype)]
        self.desc.val_type = _TORCH_VAL[str(values.dtype)]
        self.desc.row_idx = _dev_ptr(row_idx, "row_idx") if row_idx.numel() else None
        self.desc.col_idx = _dev_ptr(col_idx, "col_idx") if col_idx.numel() else None
        self.desc.values = _dev_ptr(values, "values") if values.numel() else None


class Plan:
    def __init__(self, handle, ctx, matrix):
        self.handle = handle
        self.ctx = ctx
        self.matrix = matrix   # borrowed arrays stay alive while the plan lives


def spk_solver_cfg_default() -> SolverCfg:
    cfg = SolverCfg()
    _lib.spk_solver_cfg_default(ctypes.byref(cfg))
    return cfg


def spk_init(device_id: int = 0, stream=None) -> Context:
    h = ctypes.c_void_p()
    s = None if stream is None else ctypes.c_void_p(int(stream))
    _check(_lib.spk_init(device_id, s, ctypes.byref(h)), None)
    return Context(h)


def spk_finalize(ctx: Context):
    _check(_lib.spk_finalize(ctx.handle), ctx)


def spk_csr_check(ctx: Context, A: CsrMatrix) -> int:
    v = ctypes.c_int32()
    _check(_lib.spk_csr_check(ctx.handle, ctypes.byref(A.desc), ctypes.byref(v)), ctx)
    return v.value


def spk_partition(ctx: Context, A: CsrMatrix, parts: int, split):
    if str(split.dtype) != "torch.int64" or split.numel() < parts + 1:
        raise ValueError("split must be an int64 device tensor of parts + 1 entries")
    _check(_lib.spk_partition(ctx.handle, ctypes.byref(A.desc), int(parts), _dev_ptr(split, "split")), ctx)


def spk_plan_spmv(ctx: Context, A: CsrMatrix) -> Plan:
    h = ctypes.c_void_p()
    _check(_lib.spk_plan_spmv(ctx.handle, ctypes.byref(A.desc), ctypes.byref(h)), ctx)
    return Plan(h, ctx, A)


def spk_coo_check(ctx: Context, A: CooMatrix):
    """(verdict, row_sorted)."""
    v, srt = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.spk_coo_check(ctx.handle, ctypes.byref(A.desc), ctypes.byref(v), ctypes.byref(srt)), ctx)
    return v.value, bool(srt.value)


def spk_plan_spmv_coo(ctx: Context, A: CooMatrix) -> Plan:
    h = ctypes.c_void_p()
    _check(_lib.spk_plan_spmv_coo(ctx.handle, ctypes.byref(A.desc), ctypes.byref(h)), ctx)
    return Plan(h, ctx, A)


def spk_plan_solve(ctx: Context, A: CsrMatrix, cfg: SolverCfg | None = None) -> Plan:
    h = ctypes.c_void_p()
    c = ctypes.byref(cfg) if cfg is not None else None
    _check(_lib.spk_plan_solve(ctx.handle, ctypes.byref(A.desc), c, ctypes.byref(h)), ctx)
    return Plan(h, ctx, A)


def spk_execute_spmv(plan: Plan, x, y):
    d = plan.matrix.desc
    if x.numel() < d.n_cols or y.numel() < d.n_rows:
        raise ValueError("x/y too short for the plan's matrix")
    want = "torch.float64" if d.val_type == F64 else "torch.float32"
    if str(x.dtype) != want or str(y.dtype) != want:
        raise ValueError("x and y must be %s for this matrix" % want)
    _check(_lib.spk_execute_spmv(plan.handle, _dev_ptr(x, "x"), _dev_ptr(y, "y")), plan.ctx)


def spk_execute_solve(plan: Plan, b, x) -> Log:
    d = plan.matrix.desc
    if b.numel() != d.n_rows or x.numel() != d.n_rows:
        raise ValueError("b and x must have n entries")
    if str(b.dtype) != "torch.float64" or str(x.dtype) != "torch.float64":
        raise ValueError("b and x must be float64")
    log = Log()
    _check(_lib.spk_execute_solve(plan.handle, _dev_ptr(b, "b"), _dev_ptr(x, "x"), ctypes.byref(log)), plan.ctx)
    return log


def spk_solve_noalloc(ctx: Context, A: CsrMatrix, b, x, cfg: SolverCfg | None = None) -> Log:
    """One FP64 CG solve whose workspace is the library's fixed scratch array
    (no device allocation in the call)."""
    if b.numel() != A.desc.n_rows or x.numel() != A.desc.n_rows:
        raise ValueError("b and x must have n entries")
    if str(b.dtype) != "torch.float64" or str(x.dtype) != "torch.float64":
        raise ValueError("b and x must be float64")
    log = Log()
    c = ctypes.byref(cfg) if cfg is not None else None
    _check(_lib.spk_solve_noalloc(ctx.handle, ctypes.byref(A.desc), c, _dev_ptr(b, "b"), _dev_ptr(x, "x"),
                                  ctypes.byref(log)), ctx)
    return log


def spk_noalloc_max_rows() -> int:
    return int(_lib.spk_noalloc_max_rows())


def spk_plan_history(plan: Plan) -> np.ndarray:
    count = ctypes.c_int64()
    _check(_lib.spk_plan_history(plan.handle, None, 0, ctypes.byref(count)), plan.ctx)
    out = np.empty(count.value, np.float64)
    _check(_lib.spk_plan_history(plan.handle, out.ctypes.data_as(ctypes.c_void_p), count.value,
                                 ctypes.byref(count)), plan.ctx)
    return out


def spk_plan_get_info(plan: Plan) -> dict:
    info = PlanInfo()
    _check(_lib.spk_plan_get_info(plan.handle, ctypes.byref(info)), plan.ctx)
    return info.as_dict()


def spk_plan_set_profiling(plan: Plan, on):
    """on: False/0 = off, True/1 = time every launch, k > 1 = every k-th."""
    _check(_lib.spk_plan_set_profiling(plan.handle, int(on)), plan.ctx)


def spk_plan_kernel_stats(plan: Plan):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(_lib.spk_plan_kernel_stats(plan.handle, ctypes.byref(ms), ctypes.byref(n)), plan.ctx)
    return ms.value, n.value


def spk_free(plan: Plan):
    if plan.handle:
        _check(_lib.spk_free(plan.handle), plan.ctx)
        plan.handle = None


def spk_stream_copy(ctx: Context, src, dst, nbytes: int) -> float:
    ms = ctypes.c_double()
    _check(_lib.spk_stream_copy(ctx.handle, _dev_ptr(src, "src"), _dev_ptr(dst, "dst"), int(nbytes),
                                ctypes.byref(ms)), ctx)
    return ms.value


def spk_gather_probe(ctx: Context, src, idx, dst) -> float:
    """dst[i] = src[idx[i]] with the library's gather kernel; its device time (ms)."""
    if str(src.dtype) != "torch.float64" or str(dst.dtype) != "torch.float64" or str(idx.dtype) != "torch.int32":
        raise ValueError("src and dst must be float64, idx int32")
    if dst.numel() < idx.numel():
        raise ValueError("dst shorter than idx")
    ms = ctypes.c_double()
    _check(_lib.spk_gather_probe(ctx.handle, _dev_ptr(src, "src"), int(src.numel()), _dev_ptr(idx, "idx"),
                                 int(idx.numel()), _dev_ptr(dst, "dst"), ctypes.byref(ms)), ctx)
    return ms.value


# ---------------------------------------------------------------- serving
class Server:
    def __init__(self, handle):
        self.handle = handle
        self.keep = {}   # ticket -> (matrix, b, x): kept alive until the request is done


def spk_server_request_bytes(n: int, nnz: int) -> int:
    return int(_lib.spk_server_request_bytes(int(n), int(nnz)))


def spk_server_request_bytes_prec(precision: int, n: int, nnz: int) -> int:
    return int(_lib.spk_server_request_bytes_prec(int(precision), int(n), int(nnz)))


def spk_server_request_bytes_csr(A, precision: int) -> int:
    """Workspace bytes of a request of matrix A (a CsrMatrix, or a Csr
    descriptor: only its sizes and index types are read)."""
    desc = A.desc if hasattr(A, "desc") else A
    return int(_lib.spk_server_request_bytes_csr(ctypes.byref(desc), int(precision)))


def _server_check(status, srv):
    if status != OK:
        msg = _lib.spk_server_last_error(srv.handle).decode() if srv is not None and srv.handle else ""
        raise SpkError(status, msg)


def spk_server_create(ctx: Context, hbm_budget_bytes: int, max_slots: int, cfg: SolverCfg | None = None) -> Server:
    h = ctypes.c_void_p()
    c = ctypes.byref(cfg) if cfg is not None else None
    _check(_lib.spk_server_create(ctx.handle, int(hbm_budget_bytes), int(max_slots), c, ctypes.byref(h)), ctx)
    return Server(h)


def spk_server_submit(srv: Server, A: CsrMatrix, b, x, cfg: SolverCfg | None = None) -> int:
    """Queue a solve; cfg (optional) is this request's own configuration (spk_server_submit_cfg)."""
    if b.numel() != A.desc.n_rows or x.numel() != A.desc.n_rows:
        raise ValueError("b and x must have n entries")
    if str(b.dtype) != "torch.float64" or str(x.dtype) != "torch.float64":
        raise ValueError("b and x must be float64")
    t = ctypes.c_uint64()
    if cfg is None:
        st = _lib.spk_server_submit(srv.handle, ctypes.byref(A.desc), _dev_ptr(b, "b"), _dev_ptr(x, "x"),
                                    ctypes.byref(t))
    else:
        st = _lib.spk_server_submit_cfg(srv.handle, ctypes.byref(A.desc), _dev_ptr(b, "b"), _dev_ptr(x, "x"),
                                        ctypes.byref(cfg), ctypes.byref(t))
    _server_check(st, srv)
    srv.keep[t.value] = (A, b, x)
    return t.value


def spk_server_poll(srv: Server, ticket: int):
    """Returns (done, status, Log or None, latency_ns or None) without raising on a failed request."""
    done = ctypes.c_int32()
    log = Log()
    lat = ctypes.c_int64()
    st = _lib.spk_server_poll(srv.handle, int(ticket), ctypes.byref(done), ctypes.byref(log), ctypes.byref(lat))
    if not done.value:
        if st != OK:
            _server_check(st, srv)
        return False, OK, None, None
    srv.keep.pop(int(ticket), None)
    return True, st, log, lat.value


def spk_server_drain(srv: Server):
    _server_check(_lib.spk_server_drain(srv.handle), srv)


def spk_server_get_stats(srv: Server) -> dict:
    st = ServerStats()
    _server_check(_lib.spk_server_get_stats(srv.handle, ctypes.byref(st)), srv)
    return st.as_dict()


def spk_server_destroy(srv: Server):
    if srv.handle:
        _lib.spk_server_destroy(srv.handle)
        srv.handle = None
        srv.keep.clear()
