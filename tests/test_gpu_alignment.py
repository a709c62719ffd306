"""Matrices whose value or column arrays are not 16-byte aligned.

The LDS row tiles copy a tile's values and column indices with 16-byte DMA
loads, so they need 16-byte aligned arrays.  A view of the same matrix that
starts one element into its buffer must still give the right products and
solves: its plan is tuned separately (the tuning cache tells the two apart)
and never runs the DMA tiles.  Products are compared with the FP64 oracle
within the componentwise bound 2 gamma_m (|A||x|)_i (u = 2^-53, m the row
length), and with the aligned plan's product bit for bit whenever both sum
each row in storage order (one lane per row); solves within the CG
tolerances (1e-12 relative, iteration counts within 1)."""
import numpy as np
import pytest
import torch

import inputs
import oracle
from tests.gpu_util import DEV, U64, dev_csr, gamma, rel, to_dev

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


def offset_view(t):
    """The same entries in a buffer one element longer, starting at its second element."""
    buf = torch.empty(t.numel() + 1, dtype=t.dtype, device=DEV)
    v = buf[1:]
    v.copy_(t)
    assert v.data_ptr() % 16 != 0
    return v


def misaligned(spk, M, which):
    rp, ci, va = M.tensors
    if "cols" in which:
        ci = offset_view(ci)
    if "vals" in which:
        va = offset_view(va)
    return spk.CsrMatrix(rp, ci, va, M.desc.n_rows, M.desc.n_cols)


@pytest.mark.parametrize("which", ["cols", "vals", "cols+vals"])
def test_misaligned_spmv_matches(spk, ctx, which):
    A = inputs.stencil7(50, 11)          # nnz 867,500: tuned plans
    x = inputs.vec(A.n_rows, 11, 5)
    M = dev_csr(spk, A, ptr="i32", idx="i32")
    Mm = misaligned(spk, M, which)
    xd = to_dev(x)
    ys = []
    infos = []
    for mat in (M, Mm):
        pl = spk.spk_plan_spmv(ctx, mat)
        y = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
        spk.spk_execute_spmv(pl, xd, y)
        infos.append(spk.spk_plan_get_info(pl))
        spk.spk_free(pl)
        ys.append(y.cpu().numpy())
    yo = oracle.spmv(A, x)
    m = np.diff(A.row_ptr)
    bound = 2 * gamma(m, U64) * oracle.spmv_abs(A, x)
    for y in ys:
        assert np.all(np.abs(y - yo) <= bound)
    assert infos[1]["spmv_kernel"] == 1          # never the DMA tiles
    if infos[1]["lanes"] == 1:                   # same per-row order as the tiles
        assert np.array_equal(ys[0].view(np.uint64), ys[1].view(np.uint64))


def test_misaligned_cg_and_mixed_solves(spk, ctx):
    A = inputs.stencil7(40, 12)
    b = inputs.rhs(A.n_rows, 12)
    M = dev_csr(spk, A, ptr="i32", idx="i32")
    Mm = misaligned(spk, M, "cols+vals")
    xo, res, _ = oracle.cg(A, b, tau=1e-14, max_iters=1000)
    for prec, tol in ((spk.PREC_FP64, 1e-12), (spk.PREC_MIXED_FP32, 1e-10)):
        cfg = spk.spk_solver_cfg_default()
        cfg.reduction_factor = 1e-14 if prec == spk.PREC_FP64 else 1e-12
        cfg.precision = prec
        cfg.max_iters = 5000
        for mat in (M, Mm):
            pl = spk.spk_plan_solve(ctx, mat, cfg)
            x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
            log = spk.spk_execute_solve(pl, to_dev(b), x)
            spk.spk_free(pl)
            assert log.stop_reason == spk.STOP_CONVERGED
            if prec == spk.PREC_FP64:
                assert abs(log.iterations - res.iterations) <= 1
            assert rel(x.cpu().numpy(), xo) <= tol
