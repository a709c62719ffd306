"""COO SpMV on the GPU (through spk_plan_spmv_coo) against the oracle's COO
product, plus COO validation.

Stated tolerances: FP64 |y_i - y_i^orc| <= 2 gamma_{m_i}(u) (|A||x|)_i with
u = 2^-53 and m_i the row length (each side's summation error); FP32 values
and vectors the same bound with u = 2^-24, against the oracle on the
identically rounded inputs; dyadic inputs bit-exact.  A COO plan runs the
CSR kernels over a derived row pointer, so its products equal those of the
CSR plan of the same matrix bit for bit (checked)."""
import numpy as np
import pytest
import torch

import inputs
import oracle
from tests.gpu_util import DEV, U32, U64, dev_csr, gamma, to_dev

pytestmark = pytest.mark.gpu

TIDX = {"i32": torch.int32, "i64": torch.int64}


@pytest.fixture(scope="module")
def spk():
    from paper_2510_08230_amd import spk as m
    return m


@pytest.fixture(scope="module")
def ctx(spk):
    c = spk.spk_init(0, torch.cuda.current_stream().cuda_stream)
    yield c
    spk.spk_finalize(c)


def coo_of(A):
    rows = np.repeat(np.arange(A.n_rows, dtype=np.int64), np.diff(A.row_ptr))
    return rows, A.col.astype(np.int64), A.val.copy()


def dev_coo(spk, n_rows, n_cols, rows, cols, vals, idx="i32", val=torch.float64):
    r = torch.from_numpy(np.ascontiguousarray(rows, np.int64)).to(TIDX[idx]).to(DEV)
    c = torch.from_numpy(np.ascontiguousarray(cols, np.int64)).to(TIDX[idx]).to(DEV)
    v = torch.from_numpy(np.ascontiguousarray(vals, np.float64)).to(val).to(DEV)
    return spk.CooMatrix(r, c, v, n_rows, n_cols)


def run(spk, ctx, M, x, n_rows, vtype=torch.float64, coo=True):
    pl = spk.spk_plan_spmv_coo(ctx, M) if coo else spk.spk_plan_spmv(ctx, M)
    y = torch.full((n_rows,), float("nan"), dtype=vtype, device=DEV)
    spk.spk_execute_spmv(pl, x, y)
    spk.spk_free(pl)
    return y.cpu().numpy().astype(np.float64)


def bound(n_rows, rows, cols, vals, x, u):
    m = np.maximum(np.bincount(rows, minlength=n_rows), 1)
    ab = np.zeros(n_rows)
    np.add.at(ab, rows, np.abs(vals) * np.abs(x[cols]))
    return 2 * gamma(m, u) * ab


def sparse_rows(A, keep_every=3):
    """A with every keep_every-th row (from row 1) emptied, plus empty first and last rows."""
    rows, cols, vals = coo_of(A)
    keep = (rows % keep_every != 1) & (rows != 0) & (rows != A.n_rows - 1)
    return rows[keep], cols[keep], vals[keep]


MATS = {"stencil7_46": lambda: inputs.stencil7(46, 0), "randsym_1e5": lambda: inputs.randsym(100000, 0),
        "stencil7ns_30": lambda: inputs.stencil7_ns(30, 2)}


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("idx", ["i32", "i64"])
def test_coo_fp64_within_bound_and_equal_to_csr(spk, ctx, monkeypatch, name, idx):
    monkeypatch.setenv("SPK_SPMV_KERNEL", "stream")   # one tiling for both plans
    A = MATS[name]()
    rows, cols, vals = coo_of(A)
    x = inputs.vec(A.n_cols, 1, 5)
    y = run(spk, ctx, dev_coo(spk, A.n_rows, A.n_cols, rows, cols, vals, idx), to_dev(x), A.n_rows)
    y_ref = oracle.coo_spmv(A.n_rows, rows, cols, vals, x)
    assert np.all(np.abs(y - y_ref) <= bound(A.n_rows, rows, cols, vals, x, U64))
    y_csr = run(spk, ctx, dev_csr(spk, A, "i32" if idx == "i32" else "i64", idx), to_dev(x), A.n_rows, coo=False)
    assert np.array_equal(y.view(np.uint64), y_csr.view(np.uint64))


@pytest.mark.parametrize("name", sorted(MATS))
def test_coo_fp32_within_bound(spk, ctx, name):
    A = MATS[name]()
    rows, cols, vals = sparse_rows(A)
    vals32 = vals.astype(np.float32).astype(np.float64)
    x32 = inputs.vec(A.n_cols, 2, 5).astype(np.float32).astype(np.float64)
    M = dev_coo(spk, A.n_rows, A.n_cols, rows, cols, vals32, val=torch.float32)
    y = run(spk, ctx, M, to_dev(x32, torch.float32), A.n_rows, torch.float32)
    y_ref = oracle.coo_spmv(A.n_rows, rows, cols, vals32, x32)
    # one more FP32 rounding of the stored result
    tol = bound(A.n_rows, rows, cols, vals32, x32, U32) + U32 * np.abs(y_ref)
    assert np.all(np.abs(y - y_ref) <= tol)
    empty = np.bincount(rows, minlength=A.n_rows) == 0
    assert np.all(y[empty] == 0.0)


def test_coo_dyadic_bit_exact_with_empty_rows(spk, ctx):
    A = inputs.dyadic_random(3001, 2500, 9, 7)
    rows, cols, vals = sparse_rows(A, keep_every=4)
    x = np.array([float((inputs.hash64(7, 13, j) % 17) - 8) for j in range(2500)])
    for idx in ("i32", "i64"):
        y = run(spk, ctx, dev_coo(spk, 3001, 2500, rows, cols, vals, idx), to_dev(x), 3001)
        assert np.array_equal(y, oracle.coo_spmv(3001, rows, cols, vals, x))


def test_coo_edge_cases(spk, ctx):
    # no entries at all: y = 0
    M = dev_coo(spk, 700, 5, np.zeros(0), np.zeros(0), np.zeros(0))
    y = run(spk, ctx, M, to_dev(np.ones(5)), 700)
    assert np.array_equal(y, np.zeros(700))
    # one row, many duplicates of one column
    rows = np.zeros(5000, np.int64)
    cols = np.full(5000, 2, np.int64)
    vals = np.array([inputs.unif(9, 26, k) for k in range(5000)])
    x = np.array([0.5, -1.0, 3.0])
    y = run(spk, ctx, dev_coo(spk, 1, 3, rows, cols, vals), to_dev(x), 1)
    y_ref = oracle.coo_spmv(1, rows, cols, vals, x)
    assert np.all(np.abs(y - y_ref) <= bound(1, rows, cols, vals, x, U64))
    # all entries in the last row of a tall matrix (leading empty rows)
    n = 2049
    rows = np.full(9, n - 1, np.int64)
    cols = np.arange(9, dtype=np.int64)
    vals = np.arange(1.0, 10.0)
    y = run(spk, ctx, dev_coo(spk, n, 9, rows, cols, vals), to_dev(np.ones(9)), n)
    assert y[-1] == 45.0 and not y[:-1].any()


def test_coo_validation_matches_oracle(spk, ctx):
    cases = [
        (4, 4, [0, 0, 2, 2, 3], [1, 0, 2, 3, 0]),      # ok, sorted
        (4, 4, [3, 2, 2, 0, 0], [1, 0, 2, 3, 0]),      # ok, unsorted
        (3, 4, [0, 0, 2, 2, 3], [1, 0, 2, 3, 0]),      # row out of range
        (4, 3, [0, 0, 2, 2, 3], [1, 0, 2, 3, 0]),      # column out of range
        (3, 3, [0, 1, 3], [5, 0, 0]),                  # both: rows are checked first
        (4, 4, [0, -1], [0, 0]),
    ]
    for n_rows, n_cols, r, c in cases:
        for idx in ("i32", "i64"):
            M = dev_coo(spk, n_rows, n_cols, np.array(r), np.array(c), np.ones(len(r)), idx)
            got = spk.spk_coo_check(ctx, M)
            assert got == oracle.coo_validate(n_rows, n_cols, np.array(r), np.array(c)), (n_rows, n_cols, r, c)
            if got != (0, True):
                with pytest.raises(spk.SpkError):
                    spk.spk_plan_spmv_coo(ctx, M)


def test_coo_full_size_fp32_sampled_rows(spk, ctx):
    """stencil7 N=215 as row-sorted COO with FP32 values (the paper's primary SpMV workload
    shape): 20,000 sampled rows against the oracle's definition, from the host generator."""
    N = 215
    A = inputs.stencil7(N, 1)
    rows, cols, vals = coo_of(A)
    vals32 = vals.astype(np.float32).astype(np.float64)
    x32 = inputs.vec(A.n_cols, 3, 5).astype(np.float32).astype(np.float64)
    M = dev_coo(spk, A.n_rows, A.n_cols, rows, cols, vals32, val=torch.float32)
    y = run(spk, ctx, M, to_dev(x32, torch.float32), A.n_rows, torch.float32)
    pick = np.unique(np.array([inputs.hash64(3, 27, t) % A.n_rows for t in range(20000)], np.int64))
    pick = np.concatenate([pick, [0, A.n_rows - 1]])
    for i in pick:
        a, b = int(A.row_ptr[i]), int(A.row_ptr[i + 1])
        ref = oracle.coo_spmv(1, np.zeros(b - a, np.int64), cols[a:b], vals32[a:b], x32)[0]
        ab = float(np.sum(np.abs(vals32[a:b]) * np.abs(x32[cols[a:b]])))
        assert abs(y[i] - ref) <= 2 * gamma(b - a, U32) * ab + U32 * abs(ref), i
