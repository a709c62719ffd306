"""Which CG loop a plan takes: the fused one-launch iteration up to 2^16
rows whatever the pattern, up to 2^17 rows when the pattern is banded (the
sampled row tiles hold at most 256 distinct column offsets), the
three-launch iteration otherwise; SPK_CG_FUSED forces either.  FP64 and
mixed-precision plans choose alike, and a random-pattern system in the
band solves to the oracle's solution on the loop it gets."""
import numpy as np
import pytest
import torch

import inputs
import oracle
from tests.gpu_util import DEV, dev_csr, rel, to_dev

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


CASES = [("stencil7", 46, 1), ("stencil7", 52, 0), ("randsym", 40000, 1), ("randsym", 100000, 0),
         ("randsym", 140000, 0)]


def matrix(kind, size):
    return inputs.stencil7(size, 1) if kind == "stencil7" else inputs.randsym(size, 1)


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
@pytest.mark.parametrize("kind,size,fused", CASES)
def test_loop_choice(spk, ctx, monkeypatch, kind, size, fused, precision):
    monkeypatch.delenv("SPK_CG_FUSED", raising=False)
    A = matrix(kind, size)
    cfg = spk.spk_solver_cfg_default()
    cfg.precision = spk.PREC_FP64 if precision == "fp64" else spk.PREC_MIXED_FP32
    pl = spk.spk_plan_solve(ctx, dev_csr(spk, A), cfg)
    info = spk.spk_plan_get_info(pl)
    spk.spk_free(pl)
    assert info["fused_loop"] == fused
    monkeypatch.setenv("SPK_CG_FUSED", "1")
    pl = spk.spk_plan_solve(ctx, dev_csr(spk, A), cfg)
    assert spk.spk_plan_get_info(pl)["fused_loop"] == 1
    spk.spk_free(pl)


def test_random_pattern_in_band_solves(spk, ctx, monkeypatch):
    monkeypatch.delenv("SPK_CG_FUSED", raising=False)
    A = inputs.randsym(100000, 4)
    bh = inputs.rhs(A.n_rows, 4)
    cfg = spk.spk_solver_cfg_default()
    cfg.reduction_factor = 1e-12
    pl = spk.spk_plan_solve(ctx, dev_csr(spk, A), cfg)
    assert spk.spk_plan_get_info(pl)["fused_loop"] == 0
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    log = spk.spk_execute_solve(pl, to_dev(bh), x)
    spk.spk_free(pl)
    xo, ro, _ = oracle.cg(A, bh, tau=1e-12, max_iters=1000)
    assert log.stop_reason == spk.STOP_CONVERGED
    assert abs(log.iterations - ro.iterations) <= 1
    assert rel(x.cpu().numpy(), xo) <= 1e-10
