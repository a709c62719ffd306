"""Benchmark of the sparse CG hot path on one MI355X.

Headline workload: stencil7 N=215 (n = 9,938,375 unknowns, nnz = 69,291,275),
seed 1, delta = 1, FP64 values with int32 row_ptr/col_idx, b uniform in
[-1,1), x0 = 0, solved to ||r|| <= 1e-14 ||b|| (the mid-size HBM-bound
instance).  A step is one whole solve: plan (GPU validation, tuned launch
shape, workspace) + execute (initial residual, CG iterations, true residual)
+ free, with A and b already resident in HBM.

Prints ONE JSON line.  ``value`` is updates/s = n * iterations / step time.
``roofline`` covers the dominant kernel (SpMV fused with p.q): algorithmic
bytes per launch in the format the kernel reads divided by its mean duration
from HIP events recorded around every fourth launch on the context stream
during the timed steps.  ``cpu_baseline`` is the FP64 oracle (one host core)
solving the same system to the same tolerance (capped at a bounded number of
iterations); ``error_vs_oracle`` compares the GPU's solution with the
oracle's.  The default run adds, after the timed headline steps:
  * ``mixed``: the same system by FP32 CG inside FP64 iterative refinement to
    the same tolerance (time per solve against the FP64 headline, error
    against the oracle's solution, the inner SpMV's roofline);
  * ``serving``: 256 randsym systems of log-uniform sizes through the
    continuous-batching server (saturated rate, Poisson arrivals with p50/p99
    latency), against plain FP64 solves one at a time with every plan made
    beforehand, and every result's error against the oracle;
  * ``paper_context``: the paper's own figures (other hardware), context only.
Other modes: CGS, GMRES, Jacobi PCG, the serving block alone, the large
device-generated instance and a standalone SpMV mode.
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
# HIP events bracket every PROFILE_EVERY-th launch of the dominant SpMV during
# the timed steps (every launch cost 2.8% of a C2 step; one in four, a
# quarter of that)
PROFILE_EVERY = 4

# The paper's own figures (other hardware, SuiteSparse matrices): context only.
PAPER_CONTEXT = [
    {"what": "SpMV, best of pyGinkgo CSR/COO, y = A x", "value": 150.0, "unit": "GFLOP/s (about, peak)",
     "hardware": "NVIDIA A100", "precision": "FP32", "source": "Section 6.1, GPU SpMV"},
    {"what": "CG time per iteration, pyGinkgo against CuPy", "value": 2.5, "unit": "x faster (about)",
     "hardware": "NVIDIA A100", "precision": "FP64", "source": "Section 6.2, GPU solvers"},
    {"what": "CGS against CuPy", "value": 4.0, "unit": "x faster (up to)", "hardware": "NVIDIA A100",
     "precision": "FP64", "source": "Section 6.2, GPU solvers"},
    {"what": "GMRES(30) against CuPy", "value": None, "unit": "CuPy slightly faster", "hardware": "NVIDIA A100",
     "precision": "FP64", "source": "Section 6.2, GPU solvers"},
]
PAPER_NOTE = ("context only: the paper measures other hardware on SuiteSparse matrices and prints no absolute "
              "solver times (its solver results are speedups over CuPy and SciPy)")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=215, help="stencil7 grid edge (n = N^3)")
    ap.add_argument("--pattern", choices=["stencil7", "randsym", "powerlaw"], default="stencil7",
                    help="solve-mode matrix: stencil7 N (default), randsym n or powerlaw n (randsym plus 16 hub "
                         "rows of 1e3..1e4 entries; CG only)")
    ap.add_argument("--n", type=int, default=10_000_000, help="randsym dimension")
    ap.add_argument("--delta", type=float, default=1.0,
                    help="diagonal margin: a_ii = sum |a_ij| + delta (1e-2 gives the harder system)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tau", type=float, default=1e-14)
    ap.add_argument("--solver", choices=["cg", "cgs", "gmres"], default="cg",
                    help="cgs and gmres run on the nonsymmetric stencil7 variant of the same size")
    ap.add_argument("--krylov-dim", type=int, default=30, help="GMRES restart length")
    ap.add_argument("--precond", choices=["none", "jacobi"], default="none")
    ap.add_argument("--precision", choices=["fp64", "mixed_fp32", "mixed_bf16", "mixed_fp16"], default="fp64",
                    help="fp64 solve, or an inner solve on FP32/BF16/FP16 matrix values with FP64 refinement")
    ap.add_argument("--inner", type=float, default=1e-4, help="inner reduction factor (mixed)")
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="cap on the oracle iterations of cpu_baseline (0: 60, or 12 for GMRES)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calib", action="store_true",
                    help="time the plain copy kernel (the default; kept for older command lines)")
    ap.add_argument("--no-copy-calib", action="store_true", help="skip the copy-kernel calibration")
    ap.add_argument("--no-profile", action="store_true",
                    help="time the steps without per-launch HIP events (no roofline; needed for graph/persistent)")
    ap.add_argument("--serve", action="store_true",
                    help="batched-serving run: randsym instances, Poisson arrivals, p50/p99 latency")
    ap.add_argument("--instances", type=int, default=256)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--slots", type=int, default=256)
    ap.add_argument("--load", type=float, default=0.7, help="offered load / saturated throughput")
    ap.add_argument("--no-serving", action="store_true", help="default run: skip the serving block")
    ap.add_argument("--no-mixed", action="store_true", help="default run: skip the mixed-precision block")
    ap.add_argument("--large", action="store_true",
                    help="large instance: stencil7 N=1048 generated on the device, FP32-exact values, "
                         "int64 row_ptr, FP32 CG + FP64 refinement")
    ap.add_argument("--spmv", choices=["csr", "coo"], default=None,
                    help="standalone SpMV mode y = A x (stencil7 N, seed): GFLOP/s at 2 nnz per product")
    ap.add_argument("--values", choices=["fp32", "fp64"], default="fp32", help="SpMV mode value/vector type")
    ap.add_argument("--exec", choices=["auto", "host", "graph", "persistent"], default="host",
                    help="iteration driver: host loop, captured graphs, one cooperative launch (FP64 CG; "
                         "other solves fall back to graphs), or the plan's choice")
    return ap.parse_args()


def progress(msg):
    """One line on stderr per finished phase (the JSON line stays alone on stdout)."""
    print("[bench %.1fs] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


_T0 = time.perf_counter()


def host_info():
    """CPU model, logical CPU count and memory of the host the oracle ran on."""
    info = {"nproc": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["mem_gb"] = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    return info


def index_bytes(info, n, nnz, sp):
    """Index bytes one row-tile product reads: the column index (or, with
    column codes, one byte per entry plus the 2 KiB offset table) and the row
    pointers (or, when packed, an int64 per 256-row tile and a uint16 per
    row).  sp: row-pointer width of the caller's CSR."""
    cc = int(info.get("col_codes") or 0)
    cols = nnz * 1 + 2048 if cc & 1 else nnz * 4
    rows = ((n + 255) // 256 + 1) * 8 + 2 * n if cc & 2 else (n + 1) * sp
    return cols + rows


def measured_traffic(args, N, tiling=None):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary (copy-kernel scaled), or None when
    that summary is for other kernel sources, another workload or another
    launch shape (tiling: this run's spk_plan_info)."""
    if (args.precision != "fp64" or N != 215 or args.seed != 1 or args.solver != "cg" or args.precond != "none"
            or args.pattern != "stencil7" or args.delta != 1.0):
        return None
    path = os.path.join(ROOT, "profiles", "spmv_pq_cg_fp64_stencil7_N215_traffic.json")
    if not os.path.exists(path):
        return None
    from paper_2510_08230_amd import profsum
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_digest") != profsum.kernel_digest():
        return None
    if tiling is not None and d.get("tiling") is not None:
        if any(d["tiling"][k] != tiling.get(k) for k in profsum.TILING_KEYS):
            return None
    return d["traffic_bytes"]


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: a run on several GPUs is not supported.", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve(args)
        return
    if args.large:
        large(args)
        return
    if args.spmv:
        spmv_mode(args)
        return

    import numpy as np
    import torch

    import inputs
    from paper_2510_08230_amd import spk

    dev = torch.device("cuda:0")
    N = args.N
    cgs = args.solver == "cgs"
    gm = args.solver == "gmres"
    if (cgs or args.precond != "none") and args.precision != "fp64":
        print("CGS and the Jacobi preconditioner run in FP64 only", file=sys.stderr)
        sys.exit(2)
    if args.pattern in ("randsym", "powerlaw"):
        if cgs or gm:
            print("the randsym and powerlaw patterns are symmetric: use them with CG", file=sys.stderr)
            sys.exit(2)
        A = (inputs.randsym(args.n, args.seed, delta=args.delta) if args.pattern == "randsym" else
             inputs.powerlaw(args.n, args.seed, delta=args.delta))
    elif cgs or gm:
        A = inputs.stencil7_ns(N, args.seed, delta=args.delta)
    else:
        A = inputs.stencil7(N, args.seed, delta=args.delta)
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
    cfg.exec_mode = {"auto": spk.EXEC_AUTO, "host": spk.EXEC_HOST_LOOP, "graph": spk.EXEC_GRAPH,
                     "persistent": spk.EXEC_PERSISTENT}[args.exec]
    cfg.precision = {"fp64": spk.PREC_FP64, "mixed_fp32": spk.PREC_MIXED_FP32,
                     "mixed_bf16": spk.PREC_MIXED_BF16, "mixed_fp16": spk.PREC_MIXED_FP16}[args.precision]
    cfg.inner_reduction = args.inner
    cfg.solver = spk.SOLVER_CGS if cgs else (spk.SOLVER_GMRES if gm else spk.SOLVER_CG)
    cfg.krylov_dim = args.krylov_dim
    cfg.precond = spk.PRECOND_JACOBI if args.precond == "jacobi" else spk.PRECOND_NONE
    if args.precision != "fp64":
        cfg.max_iters = 10000

    def step(profile):
        pl = spk.spk_plan_solve(ctx, M, cfg)
        if profile:
            spk.spk_plan_set_profiling(pl, PROFILE_EVERY)
        x.zero_()
        log = spk.spk_execute_solve(pl, b, x)
        stats = spk.spk_plan_kernel_stats(pl)
        info = spk.spk_plan_get_info(pl)
        spk.spk_free(pl)
        return log, stats, info

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    progress("headline warm-up done")
    t0 = time.perf_counter()
    iters, kms, klaunch = 0, 0.0, 0
    logs = []
    for _ in range(args.steps):
        log, (ms, cnt), info = step(not args.no_profile)
        iters += log.iterations
        kms += ms
        klaunch += cnt
        logs.append(log)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_per_step = wall / args.steps * 1e3
    value = n * iters / wall
    progress("headline timed steps done: %.3f ms per step" % ms_per_step)

    # index bytes: int32 columns and row pointers, or the plan's column codes
    # and packed row pointers
    idx = index_bytes(info, n, nnz, 4)
    # vectors of the dominant kernel: the SpMV reads p and writes q (2n); the
    # fused CG step reads r, q, p (gathered) and x and writes x, r, p, q (8n)
    nvec = 8 if info.get("fused_loop") else 2
    if args.precision == "fp64":
        bytes_spmv = nnz * 8 + idx + nvec * n * 8
    else:   # inner SpMV: FP32/BF16 values, int32 columns, FP32 vectors
        vb = 4 if args.precision == "mixed_fp32" else 2
        bytes_spmv = nnz * vb + idx + nvec * n * 4
    avg_ms = kms / klaunch if klaunch else None
    achieved = bytes_spmv / (avg_ms * 1e-3) / 1e9 if avg_ms else None
    last = logs[-1]
    traffic = measured_traffic(args, N, info)
    jname = "_jacobi" if args.precond == "jacobi" else ""
    dname = "" if args.delta == 1.0 else "_delta%g" % args.delta
    mname = ("%s_n%d" % (args.pattern, n)) if args.pattern in ("randsym", "powerlaw") else (
        "stencil7ns_N%d" if (cgs or gm) else "stencil7_N%d") % N
    if cgs:
        workload = "cgs%s_fp64_%s" % (jname, mname)
        spmv_kernel = "k_spmv_*<EpiCgsV>, k_spmv_*<EpiCgsR> (two SpMVs per CGS iteration)"
    elif gm:
        workload = "gmres%d%s_%s_%s" % (args.krylov_dim, jname, args.precision, mname)
        spmv_kernel = "k_spmv_*<EpiGmW> (w = A v_j / ||v_j||, one per Arnoldi step%s)" % (
            "" if args.precision == "fp64" else "; inner GMRES of the refinement")
    else:
        workload = "%s_%s_%s" % ("pcg_jacobi" if args.precond == "jacobi" else "cg", args.precision, mname)
        spmv_kernel = ("k_spmv_*<EpiFcg> (one CG step: p formed from r, q, p at every gathered column, q = A p, "
                       "x, r, p, q stored, four dot products)" if info.get("fused_loop") else
                       "k_spmv_*<EpiPq> (q = A p fused with p.q)")
    workload += dname
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
        "dtype": {"fp64": "f64", "mixed_fp32": "f32+f64", "mixed_bf16": "bf16+f32+f64",
                  "mixed_fp16": "f16+f32+f64"}[args.precision],
        "data": ("synthetic (seeded randsym: 3 uniform partners per row, symmetrised, uniform[-1,1) values, "
                 "diagonally dominant SPD, delta %g)" % args.delta if args.pattern == "randsym" else
                 "synthetic (seeded powerlaw: randsym plus 16 hub rows of 1e3..1e4 partners, symmetrised, "
                 "uniform[-1,1) values, diagonally dominant SPD, delta %g)" % args.delta if args.pattern == "powerlaw" else
                 "synthetic (seeded nonsymmetric stencil7, independent uniform[-1,1) off-diagonals, "
                 "row diagonally dominant, delta %g)" % args.delta if (cgs or gm) else
                 "synthetic (seeded stencil7, uniform[-1,1) off-diagonals, diagonally dominant SPD, "
                 "delta %g)" % args.delta),
        "config": {"workload": workload, "n": n, "nnz": nnz, "seed": args.seed,
                   "tau": args.tau, "index_types": "int32/int32", "iterations_per_solve": last.iterations,
                   "outer_iterations": last.outer_iterations,
                   "stop_reason": last.stop_reason, "rel_true_residual": last.true_resnorm / last.rhs_norm,
                   "solve_device_ms": last.elapsed_ms, "spmv_tiling": info},
        "roofline": {"bound": "hbm", "kernel": spmv_kernel,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
                     "bytes_per_launch": bytes_spmv, "avg_launch_ms": avg_ms, "launches": klaunch, "timed_every": PROFILE_EVERY},
    }
    # Rates the paper and the roofline discussion also use: nonzeros and GFLOP/s
    # (2 nnz flops per SpMV) over the timed steps, and for CG the whole
    # iteration's bytes against the floor nnz (S_v + S_i) + (n+1) S_p + 7 n S_x
    # (A once; p gathered once; x, r, p read and written once) and against the
    # vectors the loop moves (10 n S_x in three launches per iteration, 8 n S_x
    # in the one-launch fused step), over the last solve's device time.
    spmv_per_iter = 2 if cgs else 1
    spmvs = iters * spmv_per_iter
    derived = {"nnz_per_s": nnz * spmvs / wall, "gflop_per_s": 2.0 * nnz * spmvs / wall / 1e9}
    if not (cgs or gm) and last.iterations > 0:
        sv, sx = (8, 8) if args.precision == "fp64" else ((4 if args.precision == "mixed_fp32" else 2), 4)
        mat = nnz * sv + idx
        floor_b, moved_b = mat + 7 * n * sx, mat + (8 if info.get("fused_loop") else 10) * n * sx
        t_it = last.elapsed_ms * 1e-3 / last.iterations
        derived["iteration"] = {
            "floor_bytes": floor_b, "moved_bytes": moved_b, "ms": t_it * 1e3,
            "GBs_vs_floor": floor_b / t_it / 1e9, "frac_floor": floor_b / t_it / 1e9 / HBM_PEAK_GBS,
            "GBs_moved": moved_b / t_it / 1e9,
            "note": "solve device time / iterations (includes the initial and true-residual products)"}
    out["derived"] = derived
    if not args.no_copy_calib:
        nbytes = 1 << 30
        src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        best = min(spk.spk_stream_copy(ctx, src, dst, nbytes) for _ in range(5))
        cgbs = 2 * nbytes / (best * 1e-3) / 1e9
        out["copy_calib"] = {"bytes": 2 * nbytes, "ms": best, "GBs": cgbs}
        if achieved:
            out["roofline"]["frac_vs_copy"] = achieved / cgbs
        del src, dst
    if args.pattern in ("randsym", "powerlaw") and args.precision == "fp64":
        # The gathers of this matrix's SpMV without its arithmetic: dst[e] =
        # v[col[e]] over the column array in storage order (4 bytes of index
        # streamed and 8 written per gather, as the SpMV streams 4 of index and
        # 8 of value).  Its time is the ceiling the random-gather SpMV is
        # compared with, beside the HBM peak.
        src = torch.empty(n, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty(nnz, dtype=torch.float64, device=dev)
        best = min(spk.spk_gather_probe(ctx, src, ci, dst) for _ in range(5))
        out["gather_calib"] = {"gathers": nnz, "ms": best, "gathers_per_s": nnz / (best * 1e-3),
                               "note": "dst[e] = v[col[e]] over this matrix's column array (library gather "
                                       "kernel, best of 5)"}
        if avg_ms:
            out["roofline"]["frac_vs_gather"] = best / avg_ms
        del src, dst

    x_orc = None
    if not args.no_cpu_baseline:
        progress("oracle baseline")
        # The FP64 oracle on the same system with the same tolerance, capped at
        # cpu_iters iterations (a bounded sample of CPU work).  Its solution
        # also gives the GPU result's error: against the last timed solve when
        # the oracle converged, else against a GPU run of the same fixed
        # number of iterations (untimed).
        import oracle
        jac = args.precond == "jacobi"
        fn, label = oracle.cg, "CG"
        if cgs:
            fn, label = (oracle.cgs_jacobi, "CGS with Jacobi on the right") if jac else (oracle.cgs, "CGS")
        elif gm:
            fn = (lambda A_, b_, tau, max_iters: oracle.gmres(A_, b_, tau=tau, max_iters=max_iters,
                                                             m=args.krylov_dim, jacobi=jac))
            label = "GMRES(%d)%s" % (args.krylov_dim, " with Jacobi on the right" if jac else "")
        elif jac:
            fn, label = oracle.pcg_jacobi, "Jacobi PCG"
        cap = args.cpu_iters if args.cpu_iters > 0 else (12 if gm else 60)
        t0 = time.perf_counter()
        xo, res, _ = fn(A, b_h, tau=args.tau, max_iters=cap)
        dt = time.perf_counter() - t0
        if res.stop_reason == 1:
            x_gpu = x.cpu().numpy()
            compared = "the timed solve's solution vs the oracle's converged solution"
        else:
            fcfg = spk.spk_solver_cfg_default()
            for f in ("solver", "precond", "krylov_dim"):
                setattr(fcfg, f, getattr(cfg, f))
            fcfg.reduction_factor = 0.0
            fcfg.max_iters = res.iterations
            pl = spk.spk_plan_solve(ctx, M, fcfg)
            xk = torch.zeros(n, dtype=torch.float64, device=dev)
            spk.spk_execute_solve(pl, b, xk)
            spk.spk_free(pl)
            x_gpu = xk.cpu().numpy()
            compared = "GPU and oracle iterates after %d iterations (stop test off)" % res.iterations
            if args.precision != "fp64":
                compared += ("; the GPU side is the FP64 solve of the same solver (the mixed-precision "
                             "solve meets the FP64 criterion: rel_true_residual)")
        err = float(np.linalg.norm(x_gpu - xo) / np.linalg.norm(xo))
        if res.stop_reason == 1:
            x_orc = xo
        out["cpu_baseline"] = {"value": n * res.iterations / dt, "unit": "updates/s", "cores": 1,
                               "kind": "oracle", "host": host_info(),
                               "sample": "FP64 oracle %s, same system and tolerance, %d iterations (plus initial "
                                         "and true residual), %.1f s" % (label, res.iterations, dt)}
        out["error_vs_oracle"] = {"rel_2norm": err, "compared": compared,
                                  "oracle_rel_true_residual": res.true_resnorm / res.rhs_norm}
    if avg_ms:
        out["paper_context"] = {"paper": PAPER_CONTEXT, "note": PAPER_NOTE,
                                "this_run": {"spmv_fp64_gflops": 2.0 * nnz / (avg_ms * 1e-3) / 1e9,
                                             "note": "the dominant SpMV launch of this run, FP64, 2 nnz flops"}}
    plain_cg = not (cgs or gm) and args.precond == "none" and args.precision == "fp64"
    if plain_cg and not args.no_mixed:
        progress("mixed-precision block")
        try:
            out["mixed"] = mixed_block(args, ctx, M, b, x, n, nnz, ms_per_step, last, x_orc)
        except Exception as e:   # the headline line is printed whatever happens here
            out["mixed"] = {"error": repr(e)}
    spk.spk_finalize(ctx)
    if plain_cg and args.pattern == "stencil7" and not args.no_serving:
        progress("serving block")
        try:
            del M, rp, ci, va, b, x
            torch.cuda.empty_cache()
            sctx = spk.spk_init(0, torch.cuda.current_stream(dev).cuda_stream)
            out["serving"] = serving_block(args, sctx, with_oracle=not args.no_cpu_baseline)
            spk.spk_finalize(sctx)
            out["latency_s"] = out["serving"]["poisson"]["latency_s"]
        except Exception as e:
            out["serving"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


def mixed_block(args, ctx, M, b, x, n, nnz, fp64_ms, fp64_log, x_orc):
    """The same system solved by FP32 CG (FP32 values and vectors, FP64 dot
    products) inside FP64 iterative refinement to the same tolerance as the
    FP64 headline: time per whole solve (plan + solve + free, as the
    headline), updates/s on inner iterations, the inner SpMV's roofline, and
    the error against the oracle's FP64 solution."""
    import numpy as np
    import torch

    from paper_2510_08230_amd import spk

    cfg = spk.spk_solver_cfg_default()
    cfg.precision = spk.PREC_MIXED_FP32
    cfg.reduction_factor = args.tau
    cfg.inner_reduction = args.inner
    cfg.max_iters = 10000

    def step(profile):
        pl = spk.spk_plan_solve(ctx, M, cfg)
        if profile:
            spk.spk_plan_set_profiling(pl, PROFILE_EVERY)
        x.zero_()
        log = spk.spk_execute_solve(pl, b, x)
        st = spk.spk_plan_kernel_stats(pl)
        info = spk.spk_plan_get_info(pl)
        spk.spk_free(pl)
        return log, st, info

    step(False)
    steps = max(3, args.steps // 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, kms, kl = 0, 0.0, 0
    for _ in range(steps):
        log, (ms, cnt), info = step(True)
        iters += log.iterations
        kms += ms
        kl += cnt
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall / steps * 1e3
    nvec = 8 if info.get("fused_loop") else 2
    bytes_spmv = nnz * 4 + index_bytes(info, n, nnz, 4) + nvec * n * 4
    avg = kms / kl if kl else None
    ach = bytes_spmv / (avg * 1e-3) / 1e9 if avg else None
    inner_kernel = ("k_spmv_*<EpiFcg<float>> (one inner CG step on A32, FP32 vectors)" if info.get("fused_loop")
                    else "k_spmv_*<EpiPq<float>> (q = A32 p fused with p.q)")
    blk = {
        "workload": "cg_mixed_fp32_stencil7_N%d" % args.N, "dtype": "f32+f64",
        "steps": steps, "ms_per_step": ms_step, "tau": args.tau, "inner_reduction": args.inner,
        "inner_iterations": log.iterations, "outer_iterations": log.outer_iterations,
        "updates_per_s": n * iters / wall, "stop_reason": log.stop_reason,
        "rel_true_residual": log.true_resnorm / log.rhs_norm,
        "fp64_ms_per_step": fp64_ms, "fp64_iterations": fp64_log.iterations,
        "fp64_rel_true_residual": fp64_log.true_resnorm / fp64_log.rhs_norm,
        "speedup_vs_fp64": fp64_ms / ms_step,
        "inner_spmv": {"kernel": inner_kernel, "bytes_per_launch": bytes_spmv,
                       "avg_launch_ms": avg, "achieved_GBs": ach, "frac": ach / HBM_PEAK_GBS if ach else None,
                       "launches": kl, "tiling": info},
    }
    if x_orc is not None:
        xm = x.cpu().numpy()
        blk["error_vs_oracle"] = float(np.linalg.norm(xm - x_orc) / np.linalg.norm(x_orc))
        blk["equal_final_accuracy"] = bool(blk["error_vs_oracle"] <= 1e-10)
    return blk


def spmv_mode(args):
    """y = A x on stencil7 N (default 215), FP32 (the paper's SpMV benchmark type) or FP64
    values and vectors, CSR or row-sorted COO input.  A step is one product; the plan
    (validation, COO row pointer, tuning) is made once, outside the timed region."""
    import numpy as np
    import torch

    import inputs
    from paper_2510_08230_amd import spk

    dev = torch.device("cuda:0")
    N = args.N
    A = inputs.stencil7(N, args.seed)
    n, nnz = A.n_rows, A.nnz
    vt = torch.float32 if args.values == "fp32" else torch.float64
    vb = 4 if args.values == "fp32" else 8
    x_h = inputs.vec(n, args.seed, 5)
    if args.values == "fp32":
        x_h = x_h.astype(np.float32).astype(np.float64)
    va = torch.from_numpy(A.val).to(vt).to(dev)
    ci = torch.from_numpy(A.col).to(dev)
    if args.spmv == "csr":
        M = spk.CsrMatrix(torch.from_numpy(A.row_ptr).to(torch.int32).to(dev), ci, va, n, n)
    else:
        rows = torch.from_numpy(np.repeat(np.arange(n, dtype=np.int32), np.diff(A.row_ptr))).to(dev)
        M = spk.CooMatrix(rows, ci, va, n, n)
    x = torch.from_numpy(x_h).to(vt).to(dev)
    y = torch.empty(n, dtype=vt, device=dev)
    ctx = spk.spk_init(0, torch.cuda.current_stream(dev).cuda_stream)
    pl = spk.spk_plan_spmv(ctx, M) if args.spmv == "csr" else spk.spk_plan_spmv_coo(ctx, M)
    info = spk.spk_plan_get_info(pl)
    for _ in range(max(args.warmup, 1)):
        spk.spk_execute_spmv(pl, x, y)
    spk.spk_plan_set_profiling(pl, 0 if args.no_profile else PROFILE_EVERY)
    steps = max(args.steps, 1) * 10
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        spk.spk_execute_spmv(pl, x, y)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, cnt = spk.spk_plan_kernel_stats(pl)
    spk.spk_free(pl)
    spk.spk_finalize(ctx)
    # CSR tiles read the derived row pointer for COO too: (n+1) int32 (or the
    # packed form); column codes in place of the columns when derived
    bytes_spmv = nnz * vb + index_bytes(info, n, nnz, 4) + 2 * n * vb
    avg_ms = kms / cnt if cnt else None
    achieved = bytes_spmv / (avg_ms * 1e-3) / 1e9 if avg_ms else None
    out = {
        "metric": "SpMV GFLOP/s (2 nnz per product), 1 MI355X",
        "value": 2.0 * nnz * steps / wall / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1, "steps": steps, "warmup": max(args.warmup, 1),
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.values == "fp32" else "f64",
        "data": "synthetic (seeded stencil7, uniform[-1,1) values; x uniform[-1,1))",
        "config": {"workload": "spmv_%s_%s_stencil7_N%d" % (args.spmv, args.values, N), "n": n, "nnz": nnz,
                   "format": args.spmv, "index_types": "int32", "spmv_tiling": info,
                   "kernel_gflops": 2.0 * nnz / (avg_ms * 1e-3) / 1e9 if avg_ms else None},
        "roofline": {"bound": "hbm", "kernel": "k_spmv_*<EpiPlain>", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": None,
                     "bytes_per_launch": bytes_spmv, "avg_launch_ms": avg_ms, "launches": cnt, "timed_every": PROFILE_EVERY},
    }
    if not args.no_cpu_baseline:
        import oracle
        reps = 3
        t0 = time.perf_counter()
        vals = A.val.astype(np.float32).astype(np.float64) if args.values == "fp32" else A.val
        Ah = inputs.CSR(n, n, A.row_ptr, A.col, vals)
        if args.spmv == "csr":
            for _ in range(reps):
                yo = oracle.spmv(Ah, x_h)
        else:
            rows_h = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.row_ptr))
            for _ in range(reps):
                yo = oracle.coo_spmv(n, rows_h, A.col, vals, x_h)
        dt = time.perf_counter() - t0
        yg = y.cpu().numpy().astype(np.float64)
        out["error_vs_oracle"] = {"rel_2norm": float(np.linalg.norm(yg - yo) / np.linalg.norm(yo)),
                                  "max_abs": float(np.max(np.abs(yg - yo))),
                                  "compared": "last timed product vs the oracle's product of the same "
                                              "(identically rounded) inputs"}
        out["cpu_baseline"] = {"value": 2.0 * nnz * reps / dt / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
                               "host": host_info(),
                               "sample": "FP64 oracle %s product, same matrix, %d products, %.1f s"
                                         % (args.spmv.upper(), reps, dt)}
    print(json.dumps(out), flush=True)


def large(args):
    """stencil7 N (default 1048: n = 1,151,022,592, nnz = 8,050,568,320) with
    FP32-exact values generated on the device (int64 row_ptr, int32 col_idx,
    FP32 values, ~110 GB with the vectors); FP32 inner CG with FP64 dot
    products and FP64 refinement reading the same FP32 values, to
    ||b - A x|| <= 1e-12 ||b||.  Roofline: the inner SpMV+p.q kernel,
    algorithmic bytes nnz*(4+4) + (n+1)*8 + 2n*4 per launch."""
    import torch

    import inputs
    from paper_2510_08230_amd import spk

    N = 1048 if args.N == 215 else args.N
    seed = 5
    dev = torch.device("cuda:0")
    n = N ** 3
    rp, col, val = inputs.dev_stencil7(N, seed, f32x=True, val_f32=True)
    nnz = int(col.numel())
    b = inputs.dev_vec(n, seed, 2)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    M = spk.CsrMatrix(rp, col, val, n, n)
    ctx = spk.spk_init(0, torch.cuda.current_stream(dev).cuda_stream)
    cfg = spk.spk_solver_cfg_default()
    cfg.precision = spk.PREC_MIXED_FP32
    cfg.reduction_factor = 1e-12
    cfg.inner_reduction = args.inner
    cfg.max_iters = 10000
    cfg.exec_mode = {"auto": spk.EXEC_AUTO, "host": spk.EXEC_HOST_LOOP, "graph": spk.EXEC_GRAPH,
                     "persistent": spk.EXEC_PERSISTENT}[args.exec]

    def step(profile):
        pl = spk.spk_plan_solve(ctx, M, cfg)
        if profile:
            spk.spk_plan_set_profiling(pl, PROFILE_EVERY)
        x.zero_()
        log = spk.spk_execute_solve(pl, b, x)
        st = spk.spk_plan_kernel_stats(pl)
        info = spk.spk_plan_get_info(pl)
        spk.spk_free(pl)
        return log, st, info

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, kms, kl = 0, 0.0, 0
    for _ in range(args.steps):
        log, (ms, cnt), info = step(not args.no_profile)
        iters += log.iterations
        kms += ms
        kl += cnt
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    copy_calib = None
    if not args.no_copy_calib:
        # the plain copy kernel over 1 GiB each way (also the counter scale of
        # FETCH_SIZE / WRITE_SIZE runs of this mode)
        nb = 1 << 30
        src = torch.empty(nb // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        best = min(spk.spk_stream_copy(ctx, src, dst, nb) for _ in range(5))
        copy_calib = {"bytes": 2 * nb, "ms": best, "GBs": 2 * nb / (best * 1e-3) / 1e9}
        del src, dst
        # and over one FP32 vector of this size each way: the copy rate falls
        # with the buffer size (address translation over tens of GB)
        nv = n * 4 // 16 * 16
        src = torch.empty(nv // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        best = min(spk.spk_stream_copy(ctx, src, dst, nv) for _ in range(3))
        copy_calib["vector_size"] = {"bytes": 2 * nv, "ms": best, "GBs": 2 * nv / (best * 1e-3) / 1e9}
        del src, dst
    spk.spk_finalize(ctx)
    nvec = 8 if info.get("fused_loop") else 2
    bytes_spmv = nnz * 4 + index_bytes(info, n, nnz, 8) + nvec * n * 4
    avg = kms / kl if kl else None
    achieved = bytes_spmv / (avg * 1e-3) / 1e9 if avg else None
    inner_kernel = ("k_spmv_*<EpiFcg<float>> (one inner CG step on A32, FP32 vectors)" if info.get("fused_loop")
                    else "k_spmv_*<EpiPq<float>> (inner q = A32 p fused with p.q)")
    out = {
        "metric": "hot-path updates/sec and % HBM roofline, 1 MI355X; batched p50/p99 latency",
        "value": n * iters / wall, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic (seeded stencil7 generated on the device, FP32-exact values)",
        "config": {"workload": "cg_mixed_fp32_stencil7_N%d_device" % N, "n": n, "nnz": nnz, "seed": seed,
                   "tau": 1e-12, "index_types": "int64/int32", "iterations_per_solve": log.iterations,
                   "outer_iterations": log.outer_iterations, "stop_reason": log.stop_reason,
                   "rel_true_residual": log.true_resnorm / log.rhs_norm, "solve_device_ms": log.elapsed_ms,
                   "spmv_tiling": info,
                   "hbm_bytes_resident_est": (n + 1) * 8 + nnz * 8 + 2 * n * 8 + (7 if info.get("fused_loop") else 4) * n * 4},
        "roofline": {"bound": "hbm", "kernel": inner_kernel,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": None, "bytes_per_launch": bytes_spmv, "avg_launch_ms": avg, "launches": kl, "timed_every": PROFILE_EVERY},
    }
    if copy_calib:
        out["copy_calib"] = copy_calib
        if achieved:
            out["roofline"]["frac_vs_copy"] = achieved / copy_calib["GBs"]
            out["roofline"]["frac_vs_copy_vector_size"] = achieved / copy_calib["vector_size"]["GBs"]
    out["roofline"]["traffic"] = large_traffic(N, info)
    print(json.dumps(out), flush=True)


def large_traffic(N, tiling):
    """Counter traffic (bytes per inner product) of the large instance from
    its rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when that summary is
    for other kernel sources, another size or another launch shape."""
    path = os.path.join(ROOT, "profiles", "spmv_pq32_cg_mixed_fp32_stencil7_N1048_traffic.json")
    if N != 1048 or not os.path.exists(path):
        return None
    from paper_2510_08230_amd import profsum
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_digest") != profsum.kernel_digest():
        return None
    if d.get("tiling") is not None and any(d["tiling"][k] != tiling.get(k) for k in profsum.TILING_KEYS):
        return None
    return d["traffic_bytes"]


def serving_block(args, ctx, with_oracle=True):
    """The batched-serving configuration: args.instances randsym(n_i) systems,
    n_i log-uniform in [1e3, 1e6] (seed 4), b uniform, x0 = 0, solved to
    ||b - A x|| <= 1e-12 ||b|| by FP32 CG + FP64 refinement in the server.

    * closed loop (every request submitted at once) twice: the first warms
      up (graph capture, pools), the second gives the saturated rate;
    * Poisson arrivals at args.load x the saturated rate: latency p50/p99;
    * baseline: plain FP64 GPU CG solves one at a time, every plan (GPU
      validation, autotuned launch) made BEFORE the timed loop, to the same
      tolerance, saturated (back to back): the fair comparison is
      saturated serving against saturated FP64;
    * batched FP64: the same requests as FP64 CG in the server (closed loop,
      after a warm-up pass): mixed against FP64 precision, both batched;
    * accuracy: every served and every FP64 solution against the oracle's
      FP64 CG solution (tau 1e-14) of the same system, all instances, the
      oracle solves run on host threads outside every timed region.
    Returns a dict (the "serving" block of the JSON line)."""
    import numpy as np
    import torch

    import inputs
    from paper_2510_08230_amd import spk

    dev = torch.device("cuda:0")
    tau = 1e-12
    t_gen = time.perf_counter()
    hosts, rhs_h = inputs.serving_mix(args.instances, 4, 1e3, 1e6)
    gen_s = time.perf_counter() - t_gen
    progress("serving: %d instances generated in %.1f s" % (len(hosts), gen_s))
    nvec = np.array([A.n_rows for A in hosts], np.int64)
    mats = [spk.CsrMatrix(torch.from_numpy(A.row_ptr).to(torch.int32).to(dev), torch.from_numpy(A.col).to(dev),
                          torch.from_numpy(A.val).to(dev), A.n_rows, A.n_cols) for A in hosts]
    rhs = [torch.from_numpy(b).to(dev) for b in rhs_h]
    xs = [torch.zeros(int(n), dtype=torch.float64, device=dev) for n in nvec]
    cfg = spk.spk_solver_cfg_default()
    cfg.precision = spk.PREC_MIXED_FP32
    cfg.reduction_factor = tau
    cfg.inner_reduction = args.inner
    cfg.max_iters = 100000
    budget = int(args.budget_gb * (1 << 30))

    def run_pass(arrivals, pcfg=cfg):
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        srv = spk.spk_server_create(ctx, budget, args.slots, pcfg)
        t0 = time.perf_counter()
        tickets = []
        for i, M in enumerate(mats):
            if arrivals is not None:
                delay = t0 + arrivals[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            tickets.append(spk.spk_server_submit(srv, M, rhs[i], xs[i]))
        spk.spk_server_drain(srv)
        makespan = time.perf_counter() - t0
        lats, iters, outer, stops, rres = [], [], [], [], []
        for t in tickets:
            done, st, log, lat = spk.spk_server_poll(srv, t)
            assert done and st == spk.OK
            lats.append(lat * 1e-9)
            iters.append(log.iterations)
            outer.append(log.outer_iterations)
            stops.append(log.stop_reason)
            rres.append(log.true_resnorm / log.rhs_norm)
        stats = spk.spk_server_get_stats(srv)
        spk.spk_server_destroy(srv)
        return {"makespan": makespan, "lats": np.array(lats), "iters": np.array(iters), "outer": np.array(outer),
                "stops": stops, "stats": stats, "rres": rres}

    run_pass(None)                                   # warm-up
    sat = run_pass(None)
    sat_rate = len(mats) / sat["makespan"]           # solves/s, closed loop
    lam = args.load * sat_rate
    u = np.array([inputs.unif(4, 5, i) for i in range(len(mats))])
    arrivals = np.cumsum(-np.log1p(-(u + 1.0) / 2.0) / lam)
    arrivals -= arrivals[0]
    poi = run_pass(arrivals)
    progress("serving: saturated %.1f solves/s, Poisson pass done" % sat_rate)
    served = [x.cpu().numpy() for x in xs]

    # the same requests as FP64 CG in the server
    cfg64 = spk.spk_solver_cfg_default()
    cfg64.precision = spk.PREC_FP64
    cfg64.reduction_factor = tau
    cfg64.max_iters = 100000
    run_pass(None, cfg64)                            # warm-up
    sat64 = run_pass(None, cfg64)
    served64 = [x.cpu().numpy() for x in xs]
    progress("serving: batched FP64 %.1f solves/s" % (len(mats) / sat64["makespan"]))

    # baseline: plain FP64 CG, one solve at a time, plans made beforehand
    bcfg = spk.spk_solver_cfg_default()
    bcfg.reduction_factor = tau
    bcfg.max_iters = 100000
    t_plan = time.perf_counter()
    plans = [spk.spk_plan_solve(ctx, M, bcfg) for M in mats]
    plan_s = time.perf_counter() - t_plan
    for x in xs:
        x.zero_()
    spk.spk_execute_solve(plans[0], rhs[0], xs[0])   # warm-up (first solve pays one-off costs)
    xs[0].zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    base_iters, base_rres = [], []
    for i, pl in enumerate(plans):
        log = spk.spk_execute_solve(pl, rhs[i], xs[i])
        base_iters.append(log.iterations)
        base_rres.append(log.true_resnorm / log.rhs_norm)
    torch.cuda.synchronize()
    base_time = time.perf_counter() - t0
    for pl in plans:
        spk.spk_free(pl)
    fp64_sols = [x.cpu().numpy() for x in xs]
    progress("serving: FP64 baseline %.3f s (plans %.1f s outside timing)" % (base_time, plan_s))
    base_iters = np.array(base_iters)

    def pct(a, q):
        return float(np.percentile(a, q))

    # algorithmic bytes the tick SpMV moves for one pass of all requests
    nnzv = np.array([A.nnz for A in hosts], np.int64)
    tick_bytes = int(np.sum(sat["iters"] * (nnzv * 8 + (nvec + 1) * 4 + 8 * nvec)
                            + (sat["outer"] + 1) * (nnzv * 12 + (nvec + 1) * 4 + 28 * nvec)))
    # ... and for the same requests in FP64 (inner products on the FP64 values
    # and vectors; the residual writes FP64 r, p, d)
    tick_bytes64 = int(np.sum(sat64["iters"] * (nnzv * 12 + (nvec + 1) * 4 + 16 * nvec)
                              + (sat64["outer"] + 1) * (nnzv * 12 + (nvec + 1) * 4 + 40 * nvec)))

    out = {
        "workload": "serve_randsym_%d_loguniform_1e3_1e6" % len(mats),
        "data": "synthetic (seeded randsym instances: 3 uniform partners per row, symmetrised, uniform[-1,1) "
                "values, diagonally dominant SPD; sizes log-uniform in [1e3, 1e6], seed 4)",
        "instances": len(mats), "sum_n": int(nvec.sum()), "nnz_total": int(sum(A.nnz for A in hosts)),
        "tau": tau, "inner_reduction": args.inner, "dtype": "f32+f64",
        "budget_bytes": budget, "max_slots": args.slots, "offered_load": args.load,
        "arrival_rate_per_s": lam, "host_generation_s": gen_s,
        "saturated": {"makespan_s": sat["makespan"], "solves_per_s": sat_rate,
                      "updates_per_s": float(np.sum(nvec * sat["iters"])) / sat["makespan"],
                      "note": "all requests submitted at once (closed loop)"},
        "poisson": {"makespan_s": poi["makespan"], "solves_per_s": len(mats) / poi["makespan"],
                    "updates_per_s": float(np.sum(nvec * poi["iters"])) / poi["makespan"],
                    "latency_s": {"p50": pct(poi["lats"], 50), "p99": pct(poi["lats"], 99),
                                  "max": float(poi["lats"].max()), "mean": float(poi["lats"].mean())},
                    "server_stats": poi["stats"]},
        "iterations": {"inner_total": int(poi["iters"].sum()), "outer_total": int(poi["outer"].sum()),
                       "inner_max": int(poi["iters"].max())},
        "tick_spmv": {"kernel": "k_b_spmv (batched tile SpMV of a tick: FP32 inner q = A32 p, FP64 refinement "
                                "residual)",
                      "algorithmic_bytes_per_pass": tick_bytes,
                      "note": "sum over requests of inner iterations x (nnz (4+4) + (n+1) 4 + 8n) plus residual "
                              "evaluations x (nnz (8+4) + (n+1) 4 + 28n); one pass of all requests"},
        "fp64_one_at_a_time": {"seconds": base_time, "solves_per_s": len(mats) / base_time,
                               "updates_per_s": float(np.sum(nvec * base_iters)) / base_time,
                               "iterations_total": int(base_iters.sum()),
                               "plan_seconds_outside_timing": plan_s,
                               "note": "spk_execute_solve per instance back to back; every plan (validation, "
                                       "autotuned launch shape, workspace) made before the timed loop"},
        "speedup_saturated_vs_fp64": base_time / sat["makespan"],
        "fp64_batched": {"makespan_s": sat64["makespan"], "solves_per_s": len(mats) / sat64["makespan"],
                         "updates_per_s": float(np.sum(nvec * sat64["iters"])) / sat64["makespan"],
                         "iterations_total": int(sat64["iters"].sum()),
                         "outer_total": int(sat64["outer"].sum()),
                         "tick_spmv_algorithmic_bytes_per_pass": tick_bytes64,
                         "note": "the same requests as FP64 CG in the server, all submitted at once"},
        "speedup_saturated_vs_fp64_batched": sat64["makespan"] / sat["makespan"],
        "accuracy": {"served_max_rel_true_residual": float(max(poi["rres"])),
                     "fp64_max_rel_true_residual": float(max(base_rres)),
                     "fp64_batched_max_rel_true_residual": float(max(sat64["rres"])),
                     "all_converged": all(st == 1 for st in poi["stops"] + sat64["stops"])},
    }
    if with_oracle:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        t0 = time.perf_counter()
        sols = oracle.cg_many(list(zip(hosts, rhs_h)), tau=1e-14, max_iters=5000, threads=threads)
        dt = time.perf_counter() - t0
        e_srv = np.array([np.linalg.norm(a - xo) / np.linalg.norm(xo) for a, (xo, _) in zip(served, sols)])
        e_64 = np.array([np.linalg.norm(a - xo) / np.linalg.norm(xo) for a, (xo, _) in zip(fp64_sols, sols)])
        e_b64 = np.array([np.linalg.norm(a - xo) / np.linalg.norm(xo) for a, (xo, _) in zip(served64, sols)])
        o_updates = float(sum(int(A.n_rows) * r.iterations for A, (_, r) in zip(hosts, sols)))
        out["accuracy"]["served_err_vs_oracle"] = {"max": float(e_srv.max()), "p50": pct(e_srv, 50),
                                                   "p99": pct(e_srv, 99), "count": int(e_srv.size),
                                                   "within_1e-10": int(np.sum(e_srv <= 1e-10))}
        out["accuracy"]["fp64_err_vs_oracle"] = {"max": float(e_64.max()), "p50": pct(e_64, 50),
                                                 "p99": pct(e_64, 99), "count": int(e_64.size)}
        out["accuracy"]["fp64_batched_err_vs_oracle"] = {"max": float(e_b64.max()), "p50": pct(e_b64, 50),
                                                         "p99": pct(e_b64, 99), "count": int(e_b64.size)}
        out["accuracy"]["oracle"] = ("FP64 oracle CG to tau 1e-14 on every instance, %d host threads, %.1f s "
                                     "(%.3g updates/s aggregate)" % (threads, dt, o_updates / dt))
        out["accuracy"]["equal_final_accuracy"] = bool(e_srv.max() <= 1e-10 and e_64.max() <= 1e-10 and
                                                       e_b64.max() <= 1e-10)
    return out


def serve(args):
    """--serve: the serving block alone, as the line's headline (updates/s of
    the Poisson pass; p50/p99 latency beside it)."""
    import torch

    from paper_2510_08230_amd import spk

    dev = torch.device("cuda:0")
    ctx = spk.spk_init(0, torch.cuda.current_stream(dev).cuda_stream)
    blk = serving_block(args, ctx, with_oracle=not args.no_cpu_baseline)
    copy_calib = None
    if not args.no_copy_calib:
        # the plain copy kernel over 1 GiB each way (also the counter scale of
        # FETCH_SIZE / WRITE_SIZE runs of this mode)
        nb = 1 << 30
        src = torch.empty(nb // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        best = min(spk.spk_stream_copy(ctx, src, dst, nb) for _ in range(5))
        copy_calib = {"bytes": 2 * nb, "ms": best, "GBs": 2 * nb / (best * 1e-3) / 1e9}
        del src, dst
    spk.spk_finalize(ctx)
    out = {
        "metric": "hot-path updates/sec and % HBM roofline, 1 MI355X; batched p50/p99 latency",
        "value": blk["poisson"]["updates_per_s"], "unit": "updates/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": blk["poisson"]["makespan_s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": blk["data"],
        "config": {"workload": blk["workload"]},
        "latency_s": blk["poisson"]["latency_s"],
        "serving": blk,
    }
    if copy_calib:
        out["copy_calib"] = copy_calib
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
