"""The allocation-free solve (spk_solve_noalloc) against the planned solve.

Its workspace is the library's fixed per-GPU scratch array; it runs the same
kernels in the same launch shape as a plan of the same matrix (the tuned
shape an earlier plan of that shape left in the context, else the heuristic
one), so the solution equals the planned solve's bit for bit, and the
planned solve is within 1e-12 of the FP64 oracle (as in the CG tests).  Two
calls in a row, the second on a smaller system: the scratch keeps the first
call's contents, which the second must not see.  Also: a system past the
scratch limit and unsupported configurations are rejected with an error."""
import numpy as np
import pytest
import torch

import inputs
import oracle
from tests.gpu_util import dev_csr, rel, to_dev

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


def cfg_for(spk, tau=1e-14):
    cfg = spk.spk_solver_cfg_default()
    cfg.reduction_factor = tau
    cfg.max_iters = 1000
    return cfg


def planned(spk, ctx, M, b, cfg):
    pl = spk.spk_plan_solve(ctx, M, cfg)
    x = torch.zeros(M.desc.n_rows, dtype=torch.float64, device=b.device)
    log = spk.spk_execute_solve(pl, b, x)
    spk.spk_free(pl)
    return x.cpu().numpy(), log


# the second system is the smaller one; stencil7 N = 60 and 80 (216,000 and
# 512,000 rows) run three launches per iteration, the others one (the scratch
# layouts differ); all stay below the 2^22 entries from which plans build
# column codes (the allocation-free solve builds none)
@pytest.mark.parametrize("mats", [(("stencil7", 46, 0), ("stencil7", 23, 3)), (("stencil7", 60, 1), ("stencil7", 9, 2)),
                                  (("stencil7", 80, 5), ("stencil7", 50, 1)),
                                  (("randsym", 100000, 2), ("randsym", 40000, 3))])
def test_noalloc_equals_planned_twice(spk, ctx, mats, monkeypatch):
    # randsym 100,000 lies in the size band where the pattern picks the loop
    # (three launches for a random pattern), randsym 40,000 below it (fused);
    # the plans keep the default column-code choice (SPK_COL_CODES=1 would
    # give them codes on these sizes too, and with them another launch shape)
    monkeypatch.delenv("SPK_COL_CODES", raising=False)
    cfg = cfg_for(spk)
    for kind, N, seed in mats:   # the second system is the smaller one
        print("noalloc: %s %d seed=%d" % (kind, N, seed), flush=True)
        A = inputs.stencil7(N, seed) if kind == "stencil7" else inputs.randsym(N, seed)
        bh = inputs.rhs(A.n_rows, seed)
        M = dev_csr(spk, A, ptr="i32", idx="i32")
        b = to_dev(bh)
        x_plan, log_plan = planned(spk, ctx, M, b, cfg)
        x = torch.zeros(A.n_rows, dtype=torch.float64, device=b.device)
        log = spk.spk_solve_noalloc(ctx, M, b, x, cfg)
        xn = x.cpu().numpy()
        assert log.stop_reason == spk.STOP_CONVERGED
        assert log.iterations == log_plan.iterations
        assert np.array_equal(xn.view(np.uint64), x_plan.view(np.uint64))
        assert log.true_resnorm == log_plan.true_resnorm and log.rhs_norm == log_plan.rhs_norm
        xo, res, _ = oracle.cg(A, bh, tau=1e-14, max_iters=1000)
        assert abs(log.iterations - res.iterations) <= 1
        assert rel(xn, xo) <= 1e-12


def test_noalloc_initial_guess_and_cap(spk, ctx):
    """A nonzero guess and an iteration cap, against the planned solve."""
    A = inputs.stencil7(30, 4)
    bh = inputs.rhs(A.n_rows, 4)
    x0 = inputs.vec(A.n_rows, 4, 9)
    M = dev_csr(spk, A)
    b = to_dev(bh)
    cfg = cfg_for(spk)
    cfg.max_iters = 7
    pl = spk.spk_plan_solve(ctx, M, cfg)
    xp = to_dev(x0)
    lp = spk.spk_execute_solve(pl, b, xp)
    spk.spk_free(pl)
    xn = to_dev(x0)
    ln = spk.spk_solve_noalloc(ctx, M, b, xn, cfg)
    assert ln.stop_reason == spk.STOP_MAX_ITERS and ln.iterations == 7 == lp.iterations
    assert np.array_equal(xn.cpu().numpy().view(np.uint64), xp.cpu().numpy().view(np.uint64))
    xo, _, _ = oracle.cg(A, bh, x0=x0, tau=1e-14, max_iters=7)
    assert rel(xn.cpu().numpy(), xo) <= 1e-12


def test_noalloc_rejects(spk, ctx):
    limit = spk.spk_noalloc_max_rows()
    assert 2_000_000 < limit < (64 << 20) // 24
    A = inputs.stencil7(8, 0)
    M = dev_csr(spk, A)
    b = to_dev(inputs.rhs(A.n_rows, 0))
    x = torch.zeros_like(b)
    bad = cfg_for(spk)
    bad.precision = spk.PREC_MIXED_FP32
    with pytest.raises(spk.SpkError) as e:
        spk.spk_solve_noalloc(ctx, M, b, x, bad)
    assert e.value.status == spk.ERR_UNSUPPORTED
    bad = cfg_for(spk)
    bad.record_history = 1
    with pytest.raises(spk.SpkError) as e:
        spk.spk_solve_noalloc(ctx, M, b, x, bad)
    assert e.value.status == spk.ERR_UNSUPPORTED
    # one row past the limit: rejected on the host before any device work
    n = limit + 1
    rp = torch.zeros(n + 1, dtype=torch.int32, device=b.device)
    ci = torch.zeros(1, dtype=torch.int32, device=b.device)
    va = torch.zeros(1, dtype=torch.float64, device=b.device)
    big = spk.CsrMatrix(rp, ci[:0], va[:0], n, n)
    bb = torch.zeros(n, dtype=torch.float64, device=b.device)
    with pytest.raises(spk.SpkError) as e:
        spk.spk_solve_noalloc(ctx, big, bb, bb.clone(), cfg_for(spk))
    assert e.value.status == spk.ERR_INVALID_ARG
    assert "scratch limit" in spk.spk_last_error(ctx)
