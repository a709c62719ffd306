"""SpMV on the GPU against the FP64 oracle.

Tolerances: the componentwise bound |y_i - y_i^orc| <= 2 gamma_{m_i} (|A||x|)_i
(gamma_m = m u / (1 - m u), m_i the row length; u = 2^-53 for FP64, 2^-24 for
FP32 accumulation against the oracle run on the same rounded inputs), and
bit-exact on dyadic inputs where every partial sum is exact."""
import numpy as np
import pytest
import torch

import inputs
import oracle
from tests.gpu_util import DEV, U32, U64, dev_csr, gamma, to_dev

pytestmark = pytest.mark.gpu

KERNELS = ["stream", "stream-noremap", "stream,remap=3", "stream,remap=64", "stream,nt=1,remap=64,bpc=5",
           "stream,pf=0,nt=1", "vector:1", "vector:4", "vector:8", "vector:64", "vector:8,remap=16",
           "stream,remap=256,bpc=7", ""]


@pytest.fixture(scope="module")
def spk():
    from paper_2510_08230_amd import spk as m
    return m


@pytest.fixture(scope="module")
def ctx(spk):
    c = spk.spk_init(0, torch.cuda.current_stream().cuda_stream)
    yield c
    spk.spk_finalize(c)


def run_spmv(spk, ctx, M, x, vtype=torch.float64):
    pl = spk.spk_plan_spmv(ctx, M)
    y = torch.full((M.desc.n_rows,), float("nan"), dtype=vtype, device=DEV)
    spk.spk_execute_spmv(pl, x, y)
    info = spk.spk_plan_get_info(pl)
    spk.spk_free(pl)
    return y.cpu().numpy().astype(np.float64), info


def check_bound(A, x, y, u):
    y_ref = oracle.spmv(A, x)
    m = np.maximum(np.diff(A.row_ptr), 1)
    bound = 2 * gamma(m, u) * oracle.spmv_abs(A, x)
    bad = np.abs(y - y_ref) > bound
    assert not bad.any(), "first bad row %d: %r vs %r" % (np.argmax(bad), y[bad][:3], y_ref[bad][:3])


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("ptr,idx", [("i32", "i32"), ("i64", "i32"), ("i64", "i64"), ("i32", "i64")])
def test_dyadic_bit_exact(spk, ctx, monkeypatch, kernel, ptr, idx):
    monkeypatch.setenv("SPK_SPMV_KERNEL", kernel)
    A = inputs.dyadic_random(3001, 2500, 9, 4)
    x = np.array([float((inputs.hash64(4, 13, j) % 17) - 8) for j in range(2500)])
    y, _ = run_spmv(spk, ctx, dev_csr(spk, A, ptr, idx), to_dev(x))
    assert np.array_equal(y, oracle.spmv(A, x))


@pytest.mark.parametrize("kernel", KERNELS)
def test_dyadic_bit_exact_fp32(spk, ctx, monkeypatch, kernel):
    monkeypatch.setenv("SPK_SPMV_KERNEL", kernel)
    A = inputs.dyadic_random(2000, 2000, 7, 5)
    x = np.array([float((inputs.hash64(5, 13, j) % 9) - 4) for j in range(2000)])
    y, _ = run_spmv(spk, ctx, dev_csr(spk, A, val=torch.float32), to_dev(x, torch.float32), torch.float32)
    assert np.array_equal(y, oracle.spmv(A, x))


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("which", ["stencil7_46", "randsym_1e5"])
def test_c1_within_bound(spk, ctx, monkeypatch, kernel, which):
    monkeypatch.setenv("SPK_SPMV_KERNEL", kernel)
    A = inputs.stencil7(46, 0) if which == "stencil7_46" else inputs.randsym(100000, 0)
    x = inputs.vec(A.n_cols, 0, 5)
    y, _ = run_spmv(spk, ctx, dev_csr(spk, A), to_dev(x))
    check_bound(A, x, y, U64)


def _edge_matrices():
    out = {}
    out["n1"] = inputs.diagonal(np.array([3.0]))
    # empty rows at the start, middle and end, ragged tail (n not a multiple of 256)
    rp, cols, vals = [0], [], []
    n = 1000
    for i in range(n):
        if i % 7 != 3 and i not in (0, 999):
            for t in range(i % 5):
                cols.append((i * 31 + t * 17) % 1300)
                vals.append(inputs.unif(1, 20, i * 8 + t))
        rp.append(len(cols))
    out["empty_rows_rect"] = inputs.CSR(n, 1300, np.array(rp), np.array(cols, np.int32), np.array(vals))
    # long rows: tiles with more nonzeros than the LDS stage holds
    rp, cols, vals = [0], [], []
    n = 600
    for i in range(n):
        m = 3000 if i in (5, 300, 599) else (i % 9)
        for t in range(m):
            cols.append((i + 13 * t) % n)
            vals.append(inputs.unif(2, 20, i * 4096 + t))
        rp.append(len(cols))
    out["long_rows"] = inputs.CSR(n, n, np.array(rp), np.array(cols, np.int32), np.array(vals))
    out["no_nnz"] = inputs.CSR(5, 4, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0))
    out["dup_unsorted"] = inputs.CSR(3, 4, np.array([0, 3, 3, 6]), np.array([2, 0, 2, 3, 1, 0], np.int32),
                                     np.array([1.5, -2.0, 0.25, 4.0, 8.0, -1.0]))
    return out


EDGE = _edge_matrices()


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name", sorted(EDGE))
def test_edge_cases(spk, ctx, monkeypatch, kernel, name):
    monkeypatch.setenv("SPK_SPMV_KERNEL", kernel)
    A = EDGE[name]
    x = inputs.vec(A.n_cols, 3, 5)
    y, _ = run_spmv(spk, ctx, dev_csr(spk, A), to_dev(x))
    check_bound(A, x, y, U64)


@pytest.mark.parametrize("val", [torch.float32, torch.float16, torch.bfloat16])
@pytest.mark.parametrize("kernel", ["stream", "vector:8"])
def test_low_precision_values(spk, ctx, monkeypatch, kernel, val):
    """FP32 accumulation against the FP64 oracle on the identically rounded inputs."""
    monkeypatch.setenv("SPK_SPMV_KERNEL", kernel)
    A = inputs.randsym(50000, 6)
    vals_r = torch.from_numpy(A.val).to(val).to(torch.float64).numpy()
    x32 = inputs.vec(A.n_cols, 6, 5).astype(np.float32).astype(np.float64)
    Ar = inputs.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, vals_r)
    y, _ = run_spmv(spk, ctx, dev_csr(spk, A, val=val), to_dev(x32, torch.float32), torch.float32)
    # one extra rounding of the FP32 result itself
    y_ref = oracle.spmv(Ar, x32)
    m = np.maximum(np.diff(A.row_ptr), 1)
    bound = (2 * gamma(m, U32) + U32) * oracle.spmv_abs(Ar, x32)
    assert np.all(np.abs(y - y_ref) <= bound)


def test_c2_full_size_tuned(spk, ctx, monkeypatch):
    """stencil7 N=215 (n = 9,938,375), the tuned launch; every row checked."""
    monkeypatch.delenv("SPK_SPMV_KERNEL", raising=False)
    A = inputs.stencil7(215, 1)
    x = inputs.vec(A.n_cols, 1, 5)
    y, info = run_spmv(spk, ctx, dev_csr(spk, A), to_dev(x))
    print("tuned:", info)
    check_bound(A, x, y, U64)
