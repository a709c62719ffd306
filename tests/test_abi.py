"""The C-ABI library: it loads, exports every symbol include/spk.h declares,
and the binding's struct layouts match the header (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spk.h")
LIB = os.path.join(ROOT, "paper_2510_08230_amd", "libspk.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spk_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libspk.so not built"
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), "libspk.so lacks %s" % name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (spk_[a-z_]+)\b", out))
    assert set(names) <= exported


def test_binding_covers_every_declared_symbol():
    from paper_2510_08230_amd import spk
    assert set(declared_functions()) == set(spk.EXPORTED)


PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "spk.h"
#define P(T, f) printf("%s.%s %zu\n", #T, #f, offsetof(T, f));
int main(void) {
  printf("spk_csr %zu\nspk_solver_cfg %zu\nspk_log %zu\nspk_plan_info %zu\nspk_coo %zu\n",
         sizeof(spk_csr), sizeof(spk_solver_cfg), sizeof(spk_log), sizeof(spk_plan_info), sizeof(spk_coo));
  P(spk_coo, idx_type) P(spk_coo, row_idx) P(spk_coo, values)
  P(spk_csr, values) P(spk_csr, ptr_type) P(spk_solver_cfg, max_iters) P(spk_solver_cfg, reduction_factor)
  P(spk_solver_cfg, inner_reduction) P(spk_solver_cfg, max_outer) P(spk_log, elapsed_ms) P(spk_log, stop_reason)
  P(spk_plan_info, spmv_ms) P(spk_plan_info, fused_loop)
  printf("SPK_SOLVER_GMRES %d\n", (int)SPK_SOLVER_GMRES);
  P(spk_solver_cfg, krylov_dim)
  printf("SPK_SOLVER_CGS %d\nSPK_PRECOND_JACOBI %d\nSPK_EXEC_PERSISTENT %d\nSPK_PREC_MIXED_BF16 %d\n",
         (int)SPK_SOLVER_CGS, (int)SPK_PRECOND_JACOBI, (int)SPK_EXEC_PERSISTENT, (int)SPK_PREC_MIXED_BF16);
  printf("SPK_PREC_MIXED_FP16 %d\n", (int)SPK_PREC_MIXED_FP16);
  printf("spk_server_stats %zu\n", sizeof(spk_server_stats));
  P(spk_server_stats, peak_device_bytes)
  return 0;
}
"""


def test_struct_layouts_match_header(tmp_path):
    from paper_2510_08230_amd import spk
    src = tmp_path / "probe.c"
    src.write_text(PROBE)
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)], text=True).splitlines())
    assert int(got["spk_csr"]) == ctypes.sizeof(spk.Csr)
    assert int(got["spk_solver_cfg"]) == ctypes.sizeof(spk.SolverCfg)
    assert int(got["spk_log"]) == ctypes.sizeof(spk.Log)
    assert int(got["spk_plan_info"]) == ctypes.sizeof(spk.PlanInfo)
    assert int(got["spk_coo"]) == ctypes.sizeof(spk.Coo)
    assert int(got["spk_server_stats"]) == ctypes.sizeof(spk.ServerStats)
    assert int(got["spk_server_stats.peak_device_bytes"]) == spk.ServerStats.peak_device_bytes.offset
    pairs = [("spk_csr.values", spk.Csr.values), ("spk_csr.ptr_type", spk.Csr.ptr_type),
             ("spk_solver_cfg.max_iters", spk.SolverCfg.max_iters),
             ("spk_solver_cfg.reduction_factor", spk.SolverCfg.reduction_factor),
             ("spk_solver_cfg.inner_reduction", spk.SolverCfg.inner_reduction),
             ("spk_solver_cfg.max_outer", spk.SolverCfg.max_outer),
             ("spk_log.elapsed_ms", spk.Log.elapsed_ms), ("spk_log.stop_reason", spk.Log.stop_reason),
             ("spk_plan_info.spmv_ms", spk.PlanInfo.spmv_ms),
             ("spk_plan_info.fused_loop", spk.PlanInfo.fused_loop), ("spk_coo.idx_type", spk.Coo.idx_type),
             ("spk_coo.row_idx", spk.Coo.row_idx), ("spk_coo.values", spk.Coo.values)]
    for key, field in pairs:
        assert int(got[key]) == field.offset, key
    assert int(got["SPK_SOLVER_CGS"]) == spk.SOLVER_CGS and int(got["SPK_PRECOND_JACOBI"]) == spk.PRECOND_JACOBI
    assert int(got["SPK_EXEC_PERSISTENT"]) == spk.EXEC_PERSISTENT
    assert int(got["SPK_SOLVER_GMRES"]) == spk.SOLVER_GMRES
    assert int(got["spk_solver_cfg.krylov_dim"]) == spk.SolverCfg.krylov_dim.offset
    assert int(got["SPK_PREC_MIXED_BF16"]) == spk.PREC_MIXED_BF16
    assert int(got["SPK_PREC_MIXED_FP16"]) == spk.PREC_MIXED_FP16


def test_defaults_and_status_strings():
    from paper_2510_08230_amd import spk
    cfg = spk.spk_solver_cfg_default()
    assert cfg.max_iters == 1000 and cfg.reduction_factor == 1e-6    # Listings 1-2 defaults
    assert cfg.krylov_dim == 30                                         # Listings 1-2
    assert cfg.solver == spk.SOLVER_CG and cfg.precision == spk.PREC_FP64 and cfg.true_residual == 1
    assert spk.spk_status_string(spk.OK) == "SPK_OK"
    assert spk.spk_status_string(spk.ERR_INVALID_ARG) == "SPK_ERR_INVALID_ARG"


def test_enum_numbering_agrees_with_oracle():
    """Stop reasons and CSR verdicts are numbered alike on both sides (defined independently)."""
    import oracle
    from paper_2510_08230_amd import spk
    assert (spk.STOP_CONVERGED, spk.STOP_MAX_ITERS, spk.STOP_BREAKDOWN, spk.STOP_NON_FINITE) == \
        (oracle.CONVERGED, oracle.MAX_ITERS, oracle.BREAKDOWN, oracle.NON_FINITE)
    assert (spk.CSR_OK, spk.CSR_BAD_SIZE, spk.CSR_BAD_FIRST, spk.CSR_DECREASING, spk.CSR_BAD_LAST,
            spk.CSR_BAD_COLUMN) == (oracle.CSR_OK, oracle.CSR_BAD_SIZE, oracle.CSR_BAD_FIRST,
                                    oracle.CSR_DECREASING, oracle.CSR_BAD_LAST, oracle.CSR_BAD_COLUMN)


def test_binding_rejects_host_tensors():
    import torch
    from paper_2510_08230_amd import spk
    t = torch.zeros(4, dtype=torch.int64)
    with pytest.raises(ValueError):
        spk.CsrMatrix(t, t, torch.zeros(4, dtype=torch.float64), 3, 3)


def test_server_request_bytes_formula():
    """Workspace per request: 4 FP32 vectors, the FP32 value copy and 5 FP64 partials per 256-row tile,
    each piece rounded up to 256 bytes."""
    from paper_2510_08230_amd import spk

    def al(b):
        return (b + 255) // 256 * 256
    for n, nnz in [(1, 1), (1000, 7000), (256, 1792), (257, 0), (1_000_000, 7_000_000)]:
        tiles = (n + 255) // 256
        want = 4 * al(4 * n) + al(4 * max(nnz, 1)) + al(8 * 5 * max(tiles, 1))
        assert spk.spk_server_request_bytes(n, nnz) == want


def test_server_request_bytes_by_precision():
    """FP64 requests: 4 FP64 vectors and the partials, no value copy; the
    mixed figure is spk_server_request_bytes'; other precisions: 0."""
    from paper_2510_08230_amd import spk

    def al(b):
        return (b + 255) // 256 * 256
    for n, nnz in [(1, 1), (1000, 7000), (256, 1792), (257, 0), (1_000_000, 7_000_000)]:
        tiles = (n + 255) // 256
        want = 4 * al(8 * n) + al(8 * 5 * max(tiles, 1))
        assert spk.spk_server_request_bytes_prec(spk.PREC_FP64, n, nnz) == want
        assert spk.spk_server_request_bytes_prec(spk.PREC_MIXED_FP32, n, nnz) == spk.spk_server_request_bytes(n, nnz)
        assert spk.spk_server_request_bytes_prec(spk.PREC_MIXED_BF16, n, nnz) == 0


def test_server_request_bytes_by_index_types():
    """64-bit row pointers and columns add their 32-bit copies (n + 1 and nnz
    int32, each rounded up to 256 bytes); types the server does not take: 0."""
    from paper_2510_08230_amd import spk

    def al(b):
        return (b + 255) // 256 * 256
    for n, nnz in [(1, 1), (1000, 7000), (257, 0)]:
        for ptr in (spk.I32, spk.I64):
            for idx in (spk.I32, spk.I64):
                d = spk.Csr(n_rows=n, n_cols=n, nnz=nnz, ptr_type=ptr, idx_type=idx, val_type=spk.F64)
                for prec in (spk.PREC_FP64, spk.PREC_MIXED_FP32):
                    want = spk.spk_server_request_bytes_prec(prec, n, nnz)
                    want += al(4 * (n + 1)) if ptr == spk.I64 else 0
                    want += al(4 * max(nnz, 1)) if idx == spk.I64 else 0
                    assert spk.spk_server_request_bytes_csr(d, prec) == want
                assert spk.spk_server_request_bytes_csr(d, spk.PREC_MIXED_BF16) == 0
    bad = spk.Csr(n_rows=10, n_cols=10, nnz=5, ptr_type=7, idx_type=spk.I32, val_type=spk.F64)
    assert spk.spk_server_request_bytes_csr(bad, spk.PREC_FP64) == 0
