"""Row-tile launches whose grid exceeds what the kernel holds resident.

Only as many workgroups walk tiles as the kernel holds resident on the
device; the rest store zero partials.  A grid forced well above that
(16 workgroups per CU; stencil7 N = 110 has 5,199 tiles, so the grid is
not cut to the tile count) must therefore give:

* the product bit for bit (each row is summed by one lane, whatever the
  grid), on plain indices and on column codes with packed row pointers;
* solves that match the default grid's: the same iteration count and x
  within 1e-12 (the partial sums now include zeros, so the reductions may
  round differently in the last bit), for FP64 CG (three launches and the
  fused loop) and the mixed solve, whose refinement residual and
  initial/true residual products have their own epilogues and register
  counts.
"""
import numpy as np
import pytest
import torch

import inputs
from tests.gpu_util import DEV, dev_csr, rel, to_dev

pytestmark = pytest.mark.gpu

OVER = "stream,remap=64,nt=1,bpc=16"
BASE = "stream,remap=64,nt=1"


@pytest.fixture(scope="module")
def spk():
    from paper_2510_08230_amd import spk as m
    return m


@pytest.fixture(scope="module")
def ctx(spk):
    c = spk.spk_init(0, torch.cuda.current_stream().cuda_stream)
    yield c
    spk.spk_finalize(c)


def product(spk, ctx, A, x):
    pl = spk.spk_plan_spmv(ctx, dev_csr(spk, A, "i32", "i32"))
    y = torch.full((A.n_rows,), float("nan"), dtype=torch.float64, device=DEV)
    spk.spk_execute_spmv(pl, to_dev(x), y)
    info = spk.spk_plan_get_info(pl)
    spk.spk_free(pl)
    return y.cpu().numpy(), info


@pytest.mark.parametrize("codes", ["1", "0"])
def test_oversubscribed_product_bitwise(spk, ctx, monkeypatch, codes):
    A = inputs.stencil7(110, 3)
    x = inputs.vec(A.n_cols, 3, 5)
    monkeypatch.setenv("SPK_COL_CODES", codes)
    monkeypatch.setenv("SPK_SPMV_KERNEL", BASE)
    y0, i0 = product(spk, ctx, A, x)
    monkeypatch.setenv("SPK_SPMV_KERNEL", OVER)
    y1, i1 = product(spk, ctx, A, x)
    assert i1["grid"] > i0["grid"] and i1["col_codes"] == i0["col_codes"]
    assert (i0["col_codes"] == 3) == (codes == "1")
    assert np.array_equal(y0.view(np.uint64), y1.view(np.uint64))


def cg(spk, ctx, A, b, precision):
    cfg = spk.spk_solver_cfg_default()
    cfg.reduction_factor = 1e-12
    cfg.max_iters = 2000
    cfg.precision = precision
    pl = spk.spk_plan_solve(ctx, dev_csr(spk, A, "i32", "i32"), cfg)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    log = spk.spk_execute_solve(pl, to_dev(b), x)
    spk.spk_free(pl)
    return x.cpu().numpy(), log


@pytest.mark.parametrize("mode", ["fp64-3", "fp64-fused", "mixed"])
def test_oversubscribed_solves(spk, ctx, monkeypatch, mode):
    A = inputs.stencil7(110, 4)
    b = inputs.rhs(A.n_rows, 4)
    monkeypatch.setenv("SPK_COL_CODES", "1")
    monkeypatch.setenv("SPK_CG_FUSED", "1" if mode == "fp64-fused" else "0")
    prec = spk.PREC_MIXED_FP32 if mode == "mixed" else spk.PREC_FP64
    monkeypatch.setenv("SPK_SPMV_KERNEL", BASE)
    x0, l0 = cg(spk, ctx, A, b, prec)
    monkeypatch.setenv("SPK_SPMV_KERNEL", OVER)
    x1, l1 = cg(spk, ctx, A, b, prec)
    assert l0.stop_reason == spk.STOP_CONVERGED and l1.stop_reason == spk.STOP_CONVERGED
    assert l0.iterations == l1.iterations and l0.outer_iterations == l1.outer_iterations
    assert rel(x1, x0) <= 1e-12
