"""One-byte column codes (the row-tile SpMV reading each entry's column offset
from its row through a per-matrix table of at most 256 offsets).

A coded product sums every row in the same order as the plain-index kernel,
so its result must equal that kernel's bit for bit, on every value type,
index type, ragged tail and tile size; solves with and without codes must
give identical iterates, with packed row pointers (an int64 per 256-row
tile and a uint16 offset per row) and without.  The plan takes codes exactly when the pattern has
at most 256 distinct offsets c - i (checked at 256 and 257, and with an
offset that occurs in one row only, which a sampled collection misses) and
the matrix has 2^22 entries or more (SPK_COL_CODES=1, set here, builds them
at any size), and the FP64
products stay within the summation bound 2 gamma_m(u) (|A||x|)_i of the
oracle's."""
import numpy as np
import pytest
import torch

import inputs
import oracle
from tests.gpu_util import DEV, U64, dev_csr, gamma, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spk():
    from paper_2510_08230_amd import spk as m
    return m


@pytest.fixture(autouse=True)
def codes_at_any_size(monkeypatch):
    # plans build codes for matrices of 2^22 entries and more unless asked
    monkeypatch.setenv("SPK_COL_CODES", "1")


@pytest.fixture(scope="module")
def ctx(spk):
    c = spk.spk_init(0, torch.cuda.current_stream().cuda_stream)
    yield c
    spk.spk_finalize(c)


def banded(n, offsets, seed, empty_every=0, extra=None):
    """n x n matrix with entries at columns i + d for every d in offsets that
    stays in range (rows i with i % empty_every == 1 left empty; row i of
    extra also holds the offsets extra[i]), values uniform[-1, 1)."""
    rng = np.random.default_rng(seed)
    rp, cols = [0], []
    offs = np.asarray(sorted(offsets), np.int64)
    for i in range(n):
        if empty_every and i % empty_every == 1:
            rp.append(len(cols))
            continue
        c = i + (np.asarray(sorted(set(offsets) | set(extra[i])), np.int64) if extra and i in extra else offs)
        cols.extend(c[(c >= 0) & (c < n)].tolist())
        rp.append(len(cols))
    col = np.asarray(cols, np.int32)
    val = rng.uniform(-1.0, 1.0, col.size)
    return inputs.CSR(n, n, np.asarray(rp, np.int64), col, val)


def spmv(spk, ctx, M, x, n_rows, vt=torch.float64):
    pl = spk.spk_plan_spmv(ctx, M)
    info = spk.spk_plan_get_info(pl)
    y = torch.full((n_rows,), float("nan"), dtype=vt, device=DEV)
    spk.spk_execute_spmv(pl, x, y)
    torch.cuda.synchronize()
    spk.spk_free(pl)
    return y.cpu().numpy().astype(np.float64), info


MATS = {
    "stencil7_23": lambda: inputs.stencil7(23, 0),              # 12167 rows: ragged last tile
    "stencil7_46": lambda: inputs.stencil7(46, 1),
    "stencil7ns_17": lambda: inputs.stencil7_ns(17, 2),
    # 9 entries per row: 2304 per tile, past the plan's LDS row map (rows walked per thread)
    "band9": lambda: banded(3001, [-700, -64, -3, -1, 0, 1, 2, 64, 700], 3),
    "band9_empty_rows": lambda: banded(5003, [-700, -64, -3, -1, 0, 1, 2, 64, 700], 3, empty_every=7),
    "randsym_100": lambda: inputs.randsym(100, 4),              # offsets within +-99
    # offset 37 only in row 300 (second tile): a sampled collection misses it
    "band3_rare_offset": lambda: banded(5000, [-1, 0, 1], 5, extra={300: [37]}),
}


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("ptr,idx", [("i32", "i32"), ("i64", "i32"), ("i64", "i64")])
@pytest.mark.parametrize("vt", [torch.float64, torch.float32])
def test_coded_product_equals_plain_indices(spk, ctx, monkeypatch, name, ptr, idx, vt):
    A = MATS[name]()
    M = dev_csr(spk, A, ptr=ptr, idx=idx, val=vt)
    x = to_dev(inputs.vec(A.n_cols, 7, 5), vt)
    monkeypatch.setenv("SPK_SPMV_KERNEL", "stream,codes=0")
    y0, i0 = spmv(spk, ctx, M, x, A.n_rows, vt)
    monkeypatch.setenv("SPK_SPMV_KERNEL", "stream")
    y1, i1 = spmv(spk, ctx, M, x, A.n_rows, vt)          # codes and packed row pointers
    monkeypatch.setenv("SPK_SPMV_KERNEL", "stream,pack=0")
    y2, i2 = spmv(spk, ctx, M, x, A.n_rows, vt)          # codes, plain row pointers
    monkeypatch.setenv("SPK_ROW_PACK", "0")
    monkeypatch.setenv("SPK_SPMV_KERNEL", "stream")
    y3, i3 = spmv(spk, ctx, M, x, A.n_rows, vt)          # no packed rows built
    assert i0["col_codes"] == 0 and i1["col_codes"] == 3 and i2["col_codes"] == 1 and i3["col_codes"] == 1
    assert np.array_equal(y0, y1) and np.array_equal(y0, y2) and np.array_equal(y0, y3)
    if vt == torch.float64:
        xh = inputs.vec(A.n_cols, 7, 5)
        m = np.maximum(np.diff(A.row_ptr), 1)
        assert np.all(np.abs(y1 - oracle.spmv(A, xh)) <= 2 * gamma(m, U64) * oracle.spmv_abs(A, xh))


@pytest.mark.parametrize("k,coded", [(256, 3), (257, 0)])
def test_codes_taken_up_to_256_offsets(spk, ctx, monkeypatch, k, coded):
    # offsets -128 .. k-129: rows hold up to k entries, so tiles exceed the LDS
    # stage and the product takes the direct-load path
    A = banded(1500, range(-128, k - 128), 5)
    monkeypatch.setenv("SPK_SPMV_KERNEL", "stream")
    M = dev_csr(spk, A)
    x = to_dev(inputs.vec(A.n_cols, 8, 5))
    y, info = spmv(spk, ctx, M, x, A.n_rows)
    assert info["col_codes"] == coded
    monkeypatch.setenv("SPK_SPMV_KERNEL", "stream,codes=0")
    y0, _ = spmv(spk, ctx, M, x, A.n_rows)
    assert np.array_equal(y, y0)


def test_long_duplicate_row_keeps_plain_indices(spk, ctx, monkeypatch):
    # row 5 holds 70,000 duplicate entries on the diagonal (3 distinct offsets
    # overall): a row longer than 256 entries, so the plan keeps the plain
    # indices (coded kernels carry no long-row pass) and the product sums that
    # row with the whole workgroup; within the oracle's summation bound
    A = banded(600, [-1, 0, 1], 7, extra=None)
    rows = [list(A.col[A.row_ptr[i]:A.row_ptr[i + 1]]) for i in range(A.n_rows)]
    rows[5] = rows[5] + [5] * 70000
    col = np.asarray([c for r in rows for c in r], np.int32)
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    val = np.random.default_rng(8).uniform(-1.0, 1.0, col.size)
    A = inputs.CSR(600, 600, rp, col, val)
    monkeypatch.setenv("SPK_SPMV_KERNEL", "stream")
    M = dev_csr(spk, A)
    xh = inputs.vec(A.n_cols, 9, 5)
    y, info = spmv(spk, ctx, M, to_dev(xh), A.n_rows)
    assert info["col_codes"] == 0
    m = np.maximum(np.diff(A.row_ptr), 1)
    bound = 2 * gamma(m, U64) * oracle.spmv_abs(A, xh)
    assert np.all(np.abs(y - oracle.spmv(A, xh)) <= bound)
    m = np.maximum(np.diff(A.row_ptr), 1)
    assert np.all(np.abs(y - oracle.spmv(A, xh)) <= 2 * gamma(m, U64) * oracle.spmv_abs(A, xh))


@pytest.mark.parametrize("idx", ["i32", "i64"])
def test_coo_plan_with_codes_equals_plain_csr(spk, ctx, monkeypatch, idx):
    # a COO plan runs the CSR tiles over its derived row pointer, so it takes
    # codes and packed rows too
    A = MATS["band9_empty_rows"]()
    rows = np.repeat(np.arange(A.n_rows, dtype=np.int64), np.diff(A.row_ptr))
    tidx = {"i32": torch.int32, "i64": torch.int64}[idx]
    C = spk.CooMatrix(torch.from_numpy(rows).to(tidx).to(DEV),
                      torch.from_numpy(A.col.astype(np.int64)).to(tidx).to(DEV), to_dev(A.val), A.n_rows, A.n_cols)
    xh = inputs.vec(A.n_cols, 10, 5)
    monkeypatch.setenv("SPK_SPMV_KERNEL", "stream")
    pl = spk.spk_plan_spmv_coo(ctx, C)
    info = spk.spk_plan_get_info(pl)
    y = torch.full((A.n_rows,), float("nan"), dtype=torch.float64, device=DEV)
    spk.spk_execute_spmv(pl, to_dev(xh), y)
    torch.cuda.synchronize()
    spk.spk_free(pl)
    monkeypatch.setenv("SPK_SPMV_KERNEL", "stream,codes=0")
    y0, _ = spmv(spk, ctx, dev_csr(spk, A), to_dev(xh), A.n_rows)
    assert info["col_codes"] == 3
    assert np.array_equal(y.cpu().numpy(), y0)


def test_random_pattern_keeps_indices(spk, ctx):
    A = inputs.randsym(20000, 6)   # offsets spread over +-20000
    M = dev_csr(spk, A)
    y, info = spmv(spk, ctx, M, to_dev(inputs.vec(A.n_cols, 9, 5)), A.n_rows)
    assert info["col_codes"] == 0
    xh = inputs.vec(A.n_cols, 9, 5)
    m = np.maximum(np.diff(A.row_ptr), 1)
    assert np.all(np.abs(y - oracle.spmv(A, xh)) <= 2 * gamma(m, U64) * oracle.spmv_abs(A, xh))


@pytest.mark.parametrize("env,coded", [("0", 0), (None, 0), ("1", 3)])
def test_codes_by_environment_and_size(spk, ctx, monkeypatch, env, coded):
    A = inputs.stencil7(20, 0)   # 54,400 entries: below the default size for codes
    if env is None:
        monkeypatch.delenv("SPK_COL_CODES")
    else:
        monkeypatch.setenv("SPK_COL_CODES", env)
    monkeypatch.setenv("SPK_SPMV_KERNEL", "stream")
    _, info = spmv(spk, ctx, dev_csr(spk, A), to_dev(inputs.vec(A.n_cols, 1, 5)), A.n_rows)
    assert info["col_codes"] == coded


def solve(spk, ctx, A, b, precision, solver, precond=0):
    cfg = spk.spk_solver_cfg_default()
    cfg.precond = precond
    cfg.reduction_factor = 1e-12
    cfg.max_iters = 2000
    cfg.precision = precision
    cfg.solver = solver
    if precision != spk.PREC_FP64:
        cfg.inner_reduction = 1e-3
    pl = spk.spk_plan_solve(ctx, dev_csr(spk, A), cfg)
    info = spk.spk_plan_get_info(pl)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    log = spk.spk_execute_solve(pl, to_dev(b), x)
    spk.spk_free(pl)
    return x.cpu().numpy(), log, info


@pytest.mark.parametrize("case", ["cg_fp64", "cg_mixed_fp32", "cg_mixed_bf16", "gmres_fp64", "gmres_mixed_fp32",
                                  "cgs_fp64", "pcg_fp64", "gmresjac_fp64"])
def test_solves_identical_with_and_without_codes(spk, ctx, monkeypatch, case):
    solver_name, prec_name = case.split("_", 1)
    solver = {"cg": spk.SOLVER_CG, "pcg": spk.SOLVER_CG, "gmres": spk.SOLVER_GMRES, "gmresjac": spk.SOLVER_GMRES,
              "cgs": spk.SOLVER_CGS}[solver_name]
    precond = spk.PRECOND_JACOBI if solver_name in ("pcg", "gmresjac") else spk.PRECOND_NONE
    prec = {"fp64": spk.PREC_FP64, "mixed_fp32": spk.PREC_MIXED_FP32, "mixed_bf16": spk.PREC_MIXED_BF16}[prec_name]
    A = inputs.stencil7(30, 3) if solver_name in ("cg", "pcg") else inputs.stencil7_ns(30, 3)
    b = inputs.vec(A.n_rows, 3, 2)
    monkeypatch.setenv("SPK_SPMV_KERNEL", "stream,codes=0")
    x0, l0, _ = solve(spk, ctx, A, b, prec, solver, precond)
    monkeypatch.setenv("SPK_SPMV_KERNEL", "stream")
    x1, l1, i1 = solve(spk, ctx, A, b, prec, solver, precond)
    assert i1["col_codes"] == 3
    assert l0.iterations == l1.iterations and l0.outer_iterations == l1.outer_iterations
    assert np.array_equal(x0, x1)
    assert l1.converged
    assert np.linalg.norm(oracle.residual(A, b, x1)) <= 1e-11 * np.linalg.norm(b)
