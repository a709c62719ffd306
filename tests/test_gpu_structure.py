"""GPU structure work against the oracle, bit-exact: CSR verdicts and the
nnz-balanced row partition."""
import ctypes

import numpy as np
import pytest
import torch

import inputs
import oracle
from tests.gpu_util import DEV, TORCH_IDX

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spk():
    from paper_2510_08230_amd import spk as m
    return m


@pytest.fixture(scope="module")
def ctx(spk):
    c = spk.spk_init(0, torch.cuda.current_stream().cuda_stream)
    yield c
    spk.spk_finalize(c)


CASES = [
    (3, 3, [0, 2, 3, 5], [0, 2, 1, 0, 2]),
    (3, 3, [1, 2, 3, 5], [0, 2, 1, 0, 2]),
    (3, 3, [0, 3, 2, 5], [0, 2, 1, 0, 2]),
    (3, 3, [0, 2, 2, 5], [0, 2, 1, 0, 2]),
    (3, 3, [0, 2, 3, 4], [0, 2, 1, 0, 2]),
    (3, 3, [0, 2, 3, 5], [0, 3, 1, 0, 2]),
    (3, 3, [0, 2, 3, 5], [0, 2, -1, 0, 2]),
    (3, 3, [0, 3, 2, 5], [9, 9, 9, 9, 9]),
    (3, 5, [0, 2, 3, 5], [0, 4, 1, 0, 2]),
    (1, 1, [0, 0], []),
    (0, 0, [0], []),
]


@pytest.mark.parametrize("ptr,idx", [("i32", "i32"), ("i64", "i32"), ("i64", "i64"), ("i32", "i64")])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_csr_verdict_matches_oracle(spk, ctx, ptr, idx, case):
    nr, nc, rp, ci = CASES[case]
    nnz = len(ci)
    want = oracle.csr_validate(nr, nc, nnz, np.array(rp), np.array(ci, np.int64))
    M = spk.CsrMatrix(torch.tensor(rp, dtype=TORCH_IDX[ptr], device=DEV),
                      torch.tensor(ci, dtype=TORCH_IDX[idx], device=DEV),
                      torch.ones(nnz, dtype=torch.float64, device=DEV), nr, nc)
    assert spk.spk_csr_check(ctx, M) == want


def test_csr_verdict_large_random_corruption(spk, ctx):
    A = inputs.randsym(200000, 3)
    for kind in range(3):
        rp = A.row_ptr.copy()
        ci = A.col.astype(np.int64).copy()
        if kind == 0:
            rp[123457] = rp[123456] - 1          # decreasing
        elif kind == 1:
            ci[999999] = A.n_cols                # column out of range
        else:
            rp[-1] += 1                          # last != nnz
        want = oracle.csr_validate(A.n_rows, A.n_cols, A.nnz, rp, ci)
        M = spk.CsrMatrix(torch.from_numpy(rp).to(DEV), torch.from_numpy(ci).to(torch.int32).to(DEV),
                          torch.from_numpy(A.val).to(DEV), A.n_rows, A.n_cols)
        assert spk.spk_csr_check(ctx, M) == want != 0


def test_csr_bad_size_is_host_verdict(spk, ctx):
    d = spk.Csr()
    d.n_rows, d.n_cols, d.nnz = -1, 3, 0
    d.ptr_type, d.idx_type, d.val_type = spk.I64, spk.I32, spk.F64
    v = ctypes.c_int32(-7)
    st = spk._lib.spk_csr_check(ctx.handle, ctypes.byref(d), ctypes.byref(v))
    assert st == spk.OK and v.value == oracle.CSR_BAD_SIZE


def test_plan_rejects_malformed(spk, ctx):
    M = spk.CsrMatrix(torch.tensor([0, 3, 2, 5], dtype=torch.int64, device=DEV),
                      torch.tensor([0, 2, 1, 0, 2], dtype=torch.int32, device=DEV),
                      torch.ones(5, dtype=torch.float64, device=DEV), 3, 3)
    with pytest.raises(spk.SpkError) as e:
        spk.spk_plan_spmv(ctx, M)
    assert e.value.status == spk.ERR_INVALID_ARG and "row_ptr decreases" in str(e.value)


@pytest.mark.parametrize("ptr", ["i32", "i64"])
def test_partition_bit_exact(spk, ctx, ptr):
    mats = [inputs.stencil7(20, 0).row_ptr, inputs.randsym(5000, 2).row_ptr,
            np.array([0, 0, 0, 5, 5, 9, 9, 9, 20, 20, 20], np.int64), np.array([0, 0, 0], np.int64),
            inputs.stencil7(46, 0).row_ptr]
    for rp in mats:
        n = rp.size - 1
        nnz = int(rp[-1])
        ci = torch.zeros(nnz, dtype=torch.int32, device=DEV)
        M = spk.CsrMatrix(torch.from_numpy(rp).to(TORCH_IDX[ptr]).to(DEV), ci,
                          torch.zeros(nnz, dtype=torch.float64, device=DEV), n, max(n, 1))
        for P in (1, 3, 64, 1000, 4096):
            split = torch.full((P + 1,), -1, dtype=torch.int64, device=DEV)
            spk.spk_partition(ctx, M, P, split)
            assert np.array_equal(split.cpu().numpy(), oracle.partition(rp, P))
