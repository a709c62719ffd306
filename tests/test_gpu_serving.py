"""The continuous-batching solve server on the GPU.

Each request is a randsym system solved by FP32 CG with FP64 dot products
and FP64 iterative refinement to ||b - A x|| <= 1e-12 ||b||; every result is
checked against the FP64 oracle's solution (1e-10 relative, the serving
configuration's bound; derivation as for the single mixed solve: kappa_G <= 13),
and a request's solution is bitwise the same alone and in a mix.  FP64
requests (plain CG per request, the true residual confirmed at the end) are
held to the single FP64 solve's bar: the oracle's iteration count +-1 and
x within 1e-12 of its x at tau = 1e-14."""
import time

import numpy as np
import pytest
import torch

import inputs
import oracle
from tests.gpu_util import DEV, rel, to_dev

pytestmark = pytest.mark.gpu

TAU = 1e-12


@pytest.fixture(scope="module")
def spk():
    from paper_2510_08230_amd import spk as m
    return m


@pytest.fixture(scope="module")
def ctx(spk):
    c = spk.spk_init(0, torch.cuda.current_stream().cuda_stream)
    yield c
    spk.spk_finalize(c)


def make_request(spk, n, seed):
    A = inputs.randsym(n, seed)
    b = inputs.rhs(n, seed)
    M = spk.CsrMatrix(torch.from_numpy(A.row_ptr).to(torch.int32).to(DEV), torch.from_numpy(A.col).to(DEV),
                      torch.from_numpy(A.val).to(DEV), n, n)
    return A, b, M, to_dev(b), torch.zeros(n, dtype=torch.float64, device=DEV)


def server_cfg(spk, precision=None, tau=TAU):
    cfg = spk.spk_solver_cfg_default()
    cfg.precision = spk.PREC_MIXED_FP32 if precision is None else precision
    cfg.reduction_factor = tau
    cfg.inner_reduction = 1e-4
    cfg.max_iters = 20000
    return cfg


def server(spk, ctx, budget=1 << 30, slots=64, precision=None, tau=TAU):
    return spk.spk_server_create(ctx, budget, slots, server_cfg(spk, precision, tau))


def wait_all(spk, srv, tickets, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            done, st, log, lat = spk.spk_server_poll(srv, t)
            if done:
                out[t] = (st, log, lat)
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.001)
    return out


def check_oracle(A, b, x):
    xo, _, _ = oracle.cg(A, b, tau=1e-14, max_iters=5000)
    assert rel(x, xo) <= 1e-10
    assert np.linalg.norm(oracle.residual(A, b, x)) <= TAU * np.linalg.norm(b) * 1.01


def test_alone_equals_in_mix(spk, ctx):
    sizes = [3000, 777, 40000, 12345, 1000, 65536, 5000]
    reqs = [make_request(spk, n, 100 + i) for i, n in enumerate(sizes)]
    srv = server(spk, ctx)
    A0, b0, M0, bd0, x0 = reqs[2]
    t = spk.spk_server_submit(srv, M0, bd0, x0)
    res = wait_all(spk, srv, [t])
    assert res[t][0] == spk.OK and res[t][1].stop_reason == spk.STOP_CONVERGED
    alone = x0.cpu().numpy().copy()
    # the same request again, now in a mix submitted all at once
    x0.zero_()
    tickets = [spk.spk_server_submit(srv, M, bd, x) for (_, _, M, bd, x) in reqs]
    res = wait_all(spk, srv, tickets)
    spk.spk_server_destroy(srv)
    for (A, b, _, _, x), tk in zip(reqs, tickets):
        st, log, lat = res[tk]
        assert st == spk.OK and log.stop_reason == spk.STOP_CONVERGED and lat > 0
        check_oracle(A, b, x.cpu().numpy())
    assert np.array_equal(alone.view(np.uint64), x0.cpu().numpy().view(np.uint64))


def test_budget_and_slot_limits(spk, ctx):
    sizes = [20000, 30000, 25000, 22000, 28000, 21000]
    reqs = [make_request(spk, n, 200 + i) for i, n in enumerate(sizes)]
    per = max(spk.spk_server_request_bytes(n, int(r[0].nnz)) for n, r in zip(sizes, reqs))
    least = min(spk.spk_server_request_bytes(n, int(r[0].nnz)) for n, r in zip(sizes, reqs))
    budget = 2 * per + per // 2            # two of the largest fit at once, never all six
    srv = server(spk, ctx, budget=budget, slots=8)
    tickets = [spk.spk_server_submit(srv, M, bd, x) for (_, _, M, bd, x) in reqs]
    res = wait_all(spk, srv, tickets)
    stats = spk.spk_server_get_stats(srv)
    spk.spk_server_destroy(srv)
    assert stats["peak_bytes"] <= budget and stats["completed"] == len(sizes)
    assert 0 < stats["peak_device_bytes"] <= budget   # cached blocks included
    assert 2 <= stats["peak_slots"] <= budget // least < len(sizes)
    for (A, b, _, _, x), tk in zip(reqs, tickets):
        assert res[tk][0] == spk.OK
        check_oracle(A, b, x.cpu().numpy())
    srv = server(spk, ctx, slots=3)
    tickets = [spk.spk_server_submit(srv, M, bd, x) for (_, _, M, bd, x) in reqs]
    wait_all(spk, srv, tickets)
    stats = spk.spk_server_get_stats(srv)
    spk.spk_server_destroy(srv)
    assert stats["peak_slots"] <= 3 and stats["completed"] == len(sizes)


def test_arrivals_while_running(spk, ctx):
    reqs = [make_request(spk, n, 300 + i) for i, n in enumerate([200000, 150000, 3000, 9000, 4000])]
    srv = server(spk, ctx)
    t_first = [spk.spk_server_submit(srv, M, bd, x) for (_, _, M, bd, x) in reqs[:2]]
    time.sleep(0.002)
    t_late = [spk.spk_server_submit(srv, M, bd, x) for (_, _, M, bd, x) in reqs[2:]]
    res = wait_all(spk, srv, t_first + t_late)
    stats = spk.spk_server_get_stats(srv)
    spk.spk_server_destroy(srv)
    assert stats["completed"] == 5
    for (A, b, _, _, x), tk in zip(reqs, t_first + t_late):
        assert res[tk][0] == spk.OK
        check_oracle(A, b, x.cpu().numpy())


def test_rejections_and_edge_requests(spk, ctx):
    srv = server(spk, ctx, budget=1 << 20)
    A, b, M, bd, x = make_request(spk, 200000, 7)
    with pytest.raises(spk.SpkError) as e:
        spk.spk_server_submit(srv, M, bd, x)
    assert e.value.status == spk.ERR_BUDGET
    # malformed CSR: caught on the GPU before admission, reported by poll
    bad_rp = torch.tensor([0, 2, 1, 3], dtype=torch.int32, device=DEV)
    bad = spk.CsrMatrix(bad_rp, torch.tensor([0, 1, 2], dtype=torch.int32, device=DEV),
                        torch.ones(3, dtype=torch.float64, device=DEV), 3, 3)
    tb = spk.spk_server_submit(srv, bad, to_dev(np.ones(3)), torch.zeros(3, dtype=torch.float64, device=DEV))
    # b = 0: x = 0, converged
    A2, b2, M2, _, x2 = make_request(spk, 5000, 8)
    x2.fill_(3.0)
    tz = spk.spk_server_submit(srv, M2, to_dev(np.zeros(5000)), x2)
    res = wait_all(spk, srv, [tb, tz])
    spk.spk_server_destroy(srv)
    assert res[tb][0] == spk.ERR_INVALID_ARG
    assert res[tz][0] == spk.OK and res[tz][1].stop_reason == spk.STOP_CONVERGED and not x2.cpu().numpy().any()


def test_log_uniform_mix(spk, ctx):
    sizes, seeds = inputs.instances(24, 4, 1e3, 1e5)
    reqs = [make_request(spk, int(n), int(s) % 100000) for n, s in zip(sizes, seeds)]
    srv = server(spk, ctx, slots=16)
    tickets = [spk.spk_server_submit(srv, M, bd, x) for (_, _, M, bd, x) in reqs]
    res = wait_all(spk, srv, tickets)
    spk.spk_server_destroy(srv)
    for (A, b, _, _, x), tk in zip(reqs, tickets):
        assert res[tk][0] == spk.OK and res[tk][1].stop_reason == spk.STOP_CONVERGED
        check_oracle(A, b, x.cpu().numpy())


def offset_view(t):
    """The same entries in a buffer one element longer, starting at its second element."""
    buf = torch.empty(t.numel() + 1, dtype=t.dtype, device=DEV)
    v = buf[1:]
    v.copy_(t)
    assert v.data_ptr() % 16 != 0
    return v


def test_misaligned_request_equals_aligned(spk, ctx):
    """Column and value arrays off 16-byte alignment skip the LDS DMA; each
    row is summed in the same order, so the result is the same bit for bit."""
    A, b, M, bd, x = make_request(spk, 30000, 77)
    rp, ci, va = M.tensors
    Mm = spk.CsrMatrix(rp, offset_view(ci), offset_view(va), A.n_rows, A.n_cols)
    xm = torch.zeros_like(x)
    srv = server(spk, ctx)
    t1 = spk.spk_server_submit(srv, M, bd, x)
    t2 = spk.spk_server_submit(srv, Mm, bd, xm)
    res = wait_all(spk, srv, [t1, t2])
    spk.spk_server_destroy(srv)
    assert res[t1][0] == spk.OK and res[t2][0] == spk.OK
    assert res[t1][1].iterations == res[t2][1].iterations
    assert np.array_equal(x.cpu().numpy().view(np.uint64), xm.cpu().numpy().view(np.uint64))
    check_oracle(A, b, x.cpu().numpy())


def test_per_request_configuration(spk, ctx):
    """One server, one system, three requests: the server's tolerance, a
    looser one and a tighter cap; each meets its own stop test."""
    A, b, M, bd, x = make_request(spk, 50000, 78)
    x_loose, x_cap = torch.zeros_like(x), torch.zeros_like(x)
    srv = server(spk, ctx)
    loose = spk.spk_solver_cfg_default()
    loose.precision = spk.PREC_MIXED_FP32
    loose.reduction_factor = 1e-6
    loose.inner_reduction = 1e-3
    loose.max_iters = 20000
    cap = spk.spk_solver_cfg_default()
    cap.precision = spk.PREC_MIXED_FP32
    cap.reduction_factor = TAU
    cap.max_iters = 20000
    cap.max_outer = 1
    t0 = spk.spk_server_submit(srv, M, bd, x)
    t1 = spk.spk_server_submit(srv, M, bd, x_loose, loose)
    t2 = spk.spk_server_submit(srv, M, bd, x_cap, cap)
    bad = spk.spk_solver_cfg_default()       # BF16 inner precision: not what the server runs
    bad.precision = spk.PREC_MIXED_BF16
    with pytest.raises(spk.SpkError) as e:
        spk.spk_server_submit(srv, M, bd, torch.zeros_like(x), bad)
    assert e.value.status == spk.ERR_UNSUPPORTED
    res = wait_all(spk, srv, [t0, t1, t2])
    spk.spk_server_destroy(srv)
    nb = np.linalg.norm(b)
    r0 = np.linalg.norm(oracle.residual(A, b, x.cpu().numpy()))
    r1 = np.linalg.norm(oracle.residual(A, b, x_loose.cpu().numpy()))
    assert res[t0][1].stop_reason == spk.STOP_CONVERGED and r0 <= TAU * nb * 1.01
    assert res[t1][1].stop_reason == spk.STOP_CONVERGED and r1 <= 1e-6 * nb * 1.01
    assert res[t1][1].iterations < res[t0][1].iterations
    assert res[t2][1].stop_reason == spk.STOP_MAX_ITERS and res[t2][1].outer_iterations == 1


def test_fp64_requests_match_plain_cg(spk, ctx):
    """FP64 requests from x0 = 0 at tau = 1e-14 (the C2 stop test): each is
    plain CG, so its iteration count is the oracle's +-1 and x is within
    1e-12 of the oracle's; a restart from the true residual (outer
    iterations 2) may add iterations."""
    sizes = [3000, 777, 40000, 200000]
    reqs = [make_request(spk, n, 400 + i) for i, n in enumerate(sizes)]
    srv = server(spk, ctx, precision=spk.PREC_FP64, tau=1e-14)
    tickets = [spk.spk_server_submit(srv, M, bd, x) for (_, _, M, bd, x) in reqs]
    res = wait_all(spk, srv, tickets)
    stats = spk.spk_server_get_stats(srv)
    spk.spk_server_destroy(srv)
    assert stats["completed"] == len(sizes)
    for (A, b, _, _, x), tk in zip(reqs, tickets):
        st, log, _ = res[tk]
        xo, ro, _ = oracle.cg(A, b, tau=1e-14, max_iters=5000)
        print("n %d: %d iterations, %d outer (oracle %d)" % (A.n_rows, log.iterations, log.outer_iterations,
                                                            ro.iterations))
        assert st == spk.OK and log.stop_reason == spk.STOP_CONVERGED
        assert log.outer_iterations in (1, 2)
        if log.outer_iterations == 1:
            assert abs(log.iterations - ro.iterations) <= 1
        xg = x.cpu().numpy()
        assert rel(xg, xo) <= 1e-12
        assert np.linalg.norm(oracle.residual(A, b, xg)) <= 1e-14 * np.linalg.norm(b) * 1.01
        assert log.true_resnorm <= 1e-14 * np.linalg.norm(b) * 1.01


def test_fp64_edge_requests(spk, ctx):
    """FP64 requests: b = 0 gives x = 0 (converged, whatever x0 held); a
    nonzero initial guess is refined from its own residual and meets the
    stop test; max_iters = 0 stops at once with x0 untouched."""
    srv = server(spk, ctx, precision=spk.PREC_FP64)
    A, b, M, bd, x = make_request(spk, 5000, 801)
    x.fill_(3.0)
    tz = spk.spk_server_submit(srv, M, to_dev(np.zeros(5000)), x)
    A2, b2, M2, bd2, x2 = make_request(spk, 20000, 802)
    x0 = inputs.vec(20000, 802, 9)
    x2.copy_(to_dev(x0))
    tg = spk.spk_server_submit(srv, M2, bd2, x2)
    cap = server_cfg(spk, spk.PREC_FP64)
    cap.max_iters = 0
    A3, b3, M3, bd3, x3 = make_request(spk, 3000, 803)
    x3.fill_(0.5)
    tc = spk.spk_server_submit(srv, M3, bd3, x3, cap)
    res = wait_all(spk, srv, [tz, tg, tc])
    spk.spk_server_destroy(srv)
    assert res[tz][0] == spk.OK and res[tz][1].stop_reason == spk.STOP_CONVERGED and not x.cpu().numpy().any()
    assert res[tg][0] == spk.OK and res[tg][1].stop_reason == spk.STOP_CONVERGED
    check_oracle(A2, b2, x2.cpu().numpy())
    assert res[tc][0] == spk.OK and res[tc][1].stop_reason == spk.STOP_MAX_ITERS
    assert res[tc][1].iterations == 0 and np.all(x3.cpu().numpy() == 0.5)


def test_precisions_share_a_server(spk, ctx):
    """FP64 and mixed requests in one server (per-request precision): each
    result is bitwise the one the same request gets alone."""
    sizes = [3000, 40000, 12345, 65536]
    fp64 = server_cfg(spk, spk.PREC_FP64)
    mixed = server_cfg(spk)
    plan = [(n, 500 + i, fp64 if i % 2 == 0 else mixed) for i, n in enumerate(sizes)]
    plan += [(n, 600 + i, mixed if i % 2 == 0 else fp64) for i, n in enumerate(sizes)]
    reqs = [make_request(spk, n, seed) for n, seed, _ in plan]
    alone = []
    for (_, _, M, bd, x), (_, _, cfg) in zip(reqs, plan):
        srv = server(spk, ctx)
        t = spk.spk_server_submit(srv, M, bd, x, cfg)
        r = wait_all(spk, srv, [t])
        spk.spk_server_destroy(srv)
        assert r[t][0] == spk.OK and r[t][1].stop_reason == spk.STOP_CONVERGED
        alone.append(x.cpu().numpy().copy())
        x.zero_()
    srv = server(spk, ctx)
    tickets = [spk.spk_server_submit(srv, M, bd, x, cfg) for (_, _, M, bd, x), (_, _, cfg) in zip(reqs, plan)]
    res = wait_all(spk, srv, tickets)
    spk.spk_server_destroy(srv)
    for (A, b, _, _, x), tk, xa in zip(reqs, tickets, alone):
        assert res[tk][0] == spk.OK and res[tk][1].stop_reason == spk.STOP_CONVERGED
        xg = x.cpu().numpy()
        assert np.array_equal(xg.view(np.uint64), xa.view(np.uint64))
        check_oracle(A, b, xg)


def test_index_types_give_the_same_solution(spk, ctx):
    """64-bit row pointers and columns are narrowed into the request's
    workspace at admission: every index-type combination gives the int32
    request's solution bit for bit, in both precisions, in one server; the
    budget is charged the copies (spk_server_request_bytes_csr)."""
    sizes = [3000, 40000, 12345]
    combos = [(torch.int32, torch.int32), (torch.int64, torch.int64), (torch.int64, torch.int32),
              (torch.int32, torch.int64)]
    srv = server(spk, ctx)
    jobs = []
    for i, n in enumerate(sizes):
        A = inputs.randsym(n, 900 + i)
        b = inputs.rhs(n, 900 + i)
        bd = to_dev(b)
        for prec in (spk.PREC_MIXED_FP32, spk.PREC_FP64):
            for pt, it in combos:
                M = spk.CsrMatrix(torch.from_numpy(A.row_ptr).to(pt).to(DEV),
                                  torch.from_numpy(A.col.astype(np.int64)).to(it).to(DEV),
                                  torch.from_numpy(A.val).to(DEV), n, n)
                want = spk.spk_server_request_bytes_prec(prec, n, int(A.nnz))
                want += (4 * (n + 1) + 255) // 256 * 256 if pt == torch.int64 else 0
                want += (4 * max(int(A.nnz), 1) + 255) // 256 * 256 if it == torch.int64 else 0
                assert spk.spk_server_request_bytes_csr(M, prec) == want
                x = torch.zeros(n, dtype=torch.float64, device=DEV)
                t = spk.spk_server_submit(srv, M, bd, x, server_cfg(spk, prec))
                jobs.append((i, prec, (pt, it), A, b, M, x, t))
    res = wait_all(spk, srv, [j[-1] for j in jobs])
    stats = spk.spk_server_get_stats(srv)
    spk.spk_server_destroy(srv)
    assert stats["completed"] == len(jobs) and stats["failed"] == 0
    first = {}
    for i, prec, types, A, b, M, x, t in jobs:
        assert res[t][0] == spk.OK and res[t][1].stop_reason == spk.STOP_CONVERGED
        xg = x.cpu().numpy()
        key = (i, prec)
        if key not in first:
            first[key] = xg
            check_oracle(A, b, xg)
        else:
            assert np.array_equal(xg.view(np.uint64), first[key].view(np.uint64)), (key, types)


def test_fp64_budget_accounting(spk, ctx):
    """FP64 requests are charged their own workspace (4 FP64 vectors, no
    value copy) against the budget."""
    sizes = [20000, 30000, 25000, 22000]
    reqs = [make_request(spk, n, 700 + i) for i, n in enumerate(sizes)]
    per = [spk.spk_server_request_bytes_prec(spk.PREC_FP64, n, int(r[0].nnz)) for n, r in zip(sizes, reqs)]
    budget = max(per) + min(per) // 2       # one request at a time
    srv = server(spk, ctx, budget=budget, slots=8, precision=spk.PREC_FP64)
    tickets = [spk.spk_server_submit(srv, M, bd, x) for (_, _, M, bd, x) in reqs]
    res = wait_all(spk, srv, tickets)
    stats = spk.spk_server_get_stats(srv)
    spk.spk_server_destroy(srv)
    assert stats["completed"] == len(sizes) and stats["peak_slots"] == 1
    assert stats["peak_bytes"] == max(per) and stats["peak_device_bytes"] <= budget
    for (A, b, _, _, x), tk in zip(reqs, tickets):
        assert res[tk][0] == spk.OK
        check_oracle(A, b, x.cpu().numpy())


def test_full_serving_mix(spk, ctx):
    """The full serving configuration: 256 randsym instances, n log-uniform in
    [1e3, 1e6] (seed 4), all submitted at once under a 64 GB budget, every
    result within 1e-10 of the oracle's FP64 solution (tau 1e-14); then the
    same 256 requests under a 256 MB budget, which admits only a few large
    ones at a time, must give the same solutions bit for bit."""
    t0 = time.time()
    mats, rhs = inputs.serving_mix(256, 4, 1e3, 1e6)
    print("generated %d instances (sum n %d) in %.1f s" % (len(mats), sum(A.n_rows for A in mats), time.time() - t0),
          flush=True)
    reqs = []
    for A, b in zip(mats, rhs):
        M = spk.CsrMatrix(torch.from_numpy(A.row_ptr).to(torch.int32).to(DEV), torch.from_numpy(A.col).to(DEV),
                          torch.from_numpy(A.val).to(DEV), A.n_rows, A.n_cols)
        reqs.append((M, to_dev(b)))
    outs = []
    for budget, slots in ((64 << 30, 256), (256 << 20, 256)):
        xs = [torch.zeros(A.n_rows, dtype=torch.float64, device=DEV) for A in mats]
        srv = server(spk, ctx, budget=budget, slots=slots)
        tickets = [spk.spk_server_submit(srv, M, bd, x) for (M, bd), x in zip(reqs, xs)]
        res = wait_all(spk, srv, tickets, timeout=120.0)
        stats = spk.spk_server_get_stats(srv)
        spk.spk_server_destroy(srv)
        print("budget %d MB: peak slots %d, peak device bytes %d, ticks %d, %.1f s" %
              (budget >> 20, stats["peak_slots"], stats["peak_device_bytes"], stats["ticks"], time.time() - t0),
              flush=True)
        assert stats["completed"] == 256 and stats["peak_device_bytes"] <= budget
        for tk in tickets:
            assert res[tk][0] == spk.OK and res[tk][1].stop_reason == spk.STOP_CONVERGED
        outs.append([x.cpu().numpy() for x in xs])
        if budget == 256 << 20:
            assert stats["peak_slots"] < 256
    for a, b2 in zip(outs[0], outs[1]):
        assert np.array_equal(a.view(np.uint64), b2.view(np.uint64))
    sols = oracle.cg_many(list(zip(mats, rhs)), tau=1e-14, max_iters=5000)
    print("oracle solves done, %.1f s" % (time.time() - t0), flush=True)
    errs = [rel(x, xo) for x, (xo, _) in zip(outs[0], sols)]
    print("max error vs oracle %.3g" % max(errs), flush=True)
    assert max(errs) <= 1e-10
    for A, b, x in zip(mats, rhs, outs[0]):
        assert np.linalg.norm(oracle.residual(A, b, x)) <= TAU * np.linalg.norm(b) * 1.01
