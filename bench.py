"""Benchmark of the sparse CG hot path on one MI355X.

Workload: stencil7 N=215 (n = 9,938,375 unknowns, nnz = 69,291,275), seed 1,
delta = 1, FP64 values with int32 row_ptr/col_idx, b uniform in [-1,1),
x0 = 0, solved to ||r|| <= 1e-14 ||b|| (the mid-size HBM-bound instance).
A step is one whole solve: plan (GPU validation, tuned launch shape,
workspace) + execute (initial residual, CG iterations, true residual) +
free, with A and b already resident in HBM.

Prints ONE JSON line.  ``value`` is updates/s = n * iterations / step time.
``roofline`` covers the dominant kernel (SpMV fused with p.q): algorithmic
bytes per launch nnz*(8+4) + (n+1)*4 + 2n*8 divided by its mean duration from
HIP events recorded around every launch on the context stream during the
timed steps.  ``cpu_baseline`` is the FP64 oracle (one host core) on a
bounded number of iterations of the same system.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=215, help="stencil7 grid edge (n = N^3)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tau", type=float, default=1e-14)
    ap.add_argument("--cpu-iters", type=int, default=25, help="oracle iterations timed for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calib", action="store_true", help="also time the plain copy kernel")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: multi-GPU runs are not part of this build "
              "(the sharded design is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import inputs
    from paper_2510_08230_amd import spk

    dev = torch.device("cuda:0")
    N = args.N
    A = inputs.stencil7(N, args.seed)
    b_h = inputs.rhs(A.n_rows, args.seed)
    n, nnz = A.n_rows, A.nnz
    rp = torch.from_numpy(A.row_ptr).to(torch.int32).to(dev)
    ci = torch.from_numpy(A.col).to(dev)
    va = torch.from_numpy(A.val).to(dev)
    b = torch.from_numpy(b_h).to(dev)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    M = spk.CsrMatrix(rp, ci, va, n, n)
    stream = torch.cuda.current_stream(dev)
    ctx = spk.spk_init(0, stream.cuda_stream)
    cfg = spk.spk_solver_cfg_default()
    cfg.reduction_factor = args.tau
    cfg.max_iters = 1000
    cfg.exec_mode = spk.EXEC_HOST_LOOP

    def step(profile):
        pl = spk.spk_plan_solve(ctx, M, cfg)
        if profile:
            spk.spk_plan_set_profiling(pl, True)
        x.zero_()
        log = spk.spk_execute_solve(pl, b, x)
        stats = spk.spk_plan_kernel_stats(pl)
        info = spk.spk_plan_get_info(pl)
        spk.spk_free(pl)
        return log, stats, info

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, kms, klaunch = 0, 0.0, 0
    logs = []
    for _ in range(args.steps):
        log, (ms, cnt), info = step(True)
        iters += log.iterations
        kms += ms
        klaunch += cnt
        logs.append(log)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_per_step = wall / args.steps * 1e3
    value = n * iters / wall

    bytes_spmv = nnz * (8 + 4) + (n + 1) * 4 + 2 * n * 8
    avg_ms = kms / max(klaunch, 1)
    achieved = bytes_spmv / (avg_ms * 1e-3) / 1e9
    last = logs[-1]
    out = {
        "metric": "hot-path updates/sec and % HBM roofline, 1 MI355X; batched p50/p99 latency",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded stencil7, uniform[-1,1) off-diagonals, diagonally dominant SPD)",
        "config": {"workload": "cg_fp64_stencil7_N%d" % N, "n": n, "nnz": nnz, "seed": args.seed,
                   "tau": args.tau, "index_types": "int32/int32", "iterations_per_solve": last.iterations,
                   "stop_reason": last.stop_reason, "rel_true_residual": last.true_resnorm / last.rhs_norm,
                   "solve_device_ms": last.elapsed_ms, "spmv_tiling": info},
        "roofline": {"bound": "hbm", "kernel": "k_spmv_*<EpiPq> (q = A p fused with p.q)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": bytes_spmv, "avg_launch_ms": avg_ms, "launches": klaunch},
    }
    if args.copy_calib:
        nbytes = 1 << 30
        src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        best = min(spk.spk_stream_copy(ctx, src, dst, nbytes) for _ in range(5))
        out["copy_calib"] = {"bytes": 2 * nbytes, "ms": best, "GBs": 2 * nbytes / (best * 1e-3) / 1e9}
    spk.spk_finalize(ctx)

    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        _, res, _ = oracle.cg(A, b_h, tau=0.0, max_iters=args.cpu_iters)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n * res.iterations / dt, "unit": "updates/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "FP64 oracle CG, same system, %d iterations (plus initial and "
                                         "true residual), %.1f s" % (res.iterations, dt)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
