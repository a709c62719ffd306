"""Per-launch timing of the dominant SpMV (spk_plan_set_profiling): with
stride k the launches 0, k, 2k, ... that did work are timed, per solve for
solve plans and across calls for SpMV plans; the timed launches' mean
duration does not depend on the stride beyond timing noise.  A CG solve of
K iterations has K working SpMV launches in three-launch iterations and
K + 1 working steps in the fused loop (the step after the last iteration
learns of the stop before its product)."""
import math

import numpy as np
import pytest
import torch

import inputs
from tests.gpu_util import DEV, dev_csr, to_dev

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


@pytest.mark.parametrize("fused", ["1", "0"])
@pytest.mark.parametrize("every", [1, 3, 4])
def test_solve_times_every_kth_working_launch(spk, ctx, monkeypatch, every, fused):
    monkeypatch.setenv("SPK_CG_FUSED", fused)
    A = inputs.stencil7(40, 2)
    cfg = spk.spk_solver_cfg_default()
    cfg.reduction_factor = 1e-10
    pl = spk.spk_plan_solve(ctx, dev_csr(spk, A), cfg)
    assert spk.spk_plan_get_info(pl)["fused_loop"] == int(fused)
    spk.spk_plan_set_profiling(pl, every)
    iters = []
    for _ in range(2):
        x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
        iters.append(spk.spk_execute_solve(pl, to_dev(inputs.vec(A.n_rows, 2, 2)), x).iterations)
    ms, count = spk.spk_plan_kernel_stats(pl)
    spk.spk_free(pl)
    assert iters[0] == iters[1] > 0
    working = iters[0] + (1 if fused == "1" else 0)
    assert count == 2 * math.ceil(working / every)
    assert ms > 0.0


@pytest.mark.parametrize("every", [1, 3])
def test_gmres_times_only_working_arnoldi_steps(spk, ctx, every):
    """GMRES(10) over several restarts: its last cycle stops early and the
    Arnoldi launches enqueued after the stop find nothing to do; only the
    working ones are timed (ceil(steps / k) of them)."""
    A = inputs.stencil7_ns(24, 3)
    cfg = spk.spk_solver_cfg_default()
    cfg.solver = spk.SOLVER_GMRES
    cfg.krylov_dim = 10
    cfg.reduction_factor = 1e-10
    pl = spk.spk_plan_solve(ctx, dev_csr(spk, A), cfg)
    spk.spk_plan_set_profiling(pl, every)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    log = spk.spk_execute_solve(pl, to_dev(inputs.vec(A.n_rows, 2, 2)), x)
    ms, count = spk.spk_plan_kernel_stats(pl)
    spk.spk_free(pl)
    assert log.stop_reason == spk.STOP_CONVERGED and log.iterations > 10 and log.iterations % 10 != 0
    assert count == math.ceil(log.iterations / every)
    assert ms > 0.0


def test_spmv_plan_counts_across_calls(spk, ctx):
    A = inputs.stencil7(30, 1)
    pl = spk.spk_plan_spmv(ctx, dev_csr(spk, A))
    spk.spk_plan_set_profiling(pl, 4)
    x = to_dev(inputs.vec(A.n_cols, 1, 5))
    y = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
    for _ in range(10):
        spk.spk_execute_spmv(pl, x, y)
    ms, count = spk.spk_plan_kernel_stats(pl)
    assert count == 3 and ms > 0.0          # calls 0, 4 and 8
    spk.spk_plan_set_profiling(pl, 0)        # off: nothing more is timed
    spk.spk_execute_spmv(pl, x, y)
    ms0, count0 = spk.spk_plan_kernel_stats(pl)
    assert count0 == 0 and ms0 == 0.0
    spk.spk_free(pl)
    assert np.all(np.isfinite(y.cpu().numpy()))
