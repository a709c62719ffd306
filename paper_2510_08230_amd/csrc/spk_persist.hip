// Persistent solves: the whole CG solve in one cooperative launch, every
// workgroup resident, the iterations separated by grid barriers instead of
// kernel boundaries.  Each iteration is the fused CG step of spk_fcg.h (one
// pass: the SpMV forms p from the previous r, q and p and updates x, r, p),
// so an iteration costs one barrier.
//
//   FP64 CG:   initial residual | barrier | steps k = 0, 1, ... each followed
//              by a barrier | the true residual at exit.
//   Mixed:     repeat { FP64 refinement residual r = b - A x (the outer
//              values) | barrier | FP32 inner steps on A32 d = fl32(r), each
//              followed by a barrier | x += d | barrier } until
//              ||b - A x|| <= tau ||b|| (or a cap), as the host-driven mixed
//              solve does.
//
// After a barrier every workgroup sums the same partials in the same order, so
// all take identical decisions and leave their loops together; workgroup 0
// mirrors the results for the host.  The barrier: one agent-scope
// acquire-release arrival per workgroup on a counter, relaxed polling of a
// generation word, an acquire fence once it moves; the release writes this
// workgroup's stores back to memory for every XCD, the acquire drops stale
// lines.  A wait longer than the wall-clock limit sets the error word and
// every workgroup leaves, so the launch always ends.
#include "spk_fcg.h"
#include "spk_launch.h"
#include "spk_spmv.h"

#include <type_traits>

namespace spk {
namespace {

using namespace dev;
using namespace tile;

// Grid-wide barrier; false once any workgroup has timed out (then leave).
__device__ __forceinline__ bool grid_sync(unsigned *bar, unsigned &gen, uint64_t spin_ticks) {
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
        if (ok) {
            const unsigned g0 = gen;
            const unsigned prev = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (prev == gridDim.x - 1) {
                __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&bar[1], g0 + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
                    if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    if (wall_clock64() - t0 > spin_ticks) {
                        __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                }
            }
            gen = g0 + 1;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// The epilogue of a fused step: its row work and where its partials go.
template <typename T>
struct EpiStep : fcg::Rows<T> {
    double *part;   // the step's partial set
    __device__ bool skip() const { return false; }
    __device__ void finish() { block_partial<4>(this->acc, part); }
};

// Partials of ||b - A x||^2.
struct EpiResid {
    const double *b;
    double *part;
    double acc;
    __device__ bool skip() const { return false; }
    __device__ void row(int64_t i, double s) {
        const double ri = b[i] - s;
        acc = fma(ri, ri, acc);
    }
    __device__ void finish() {
        double v[1] = {acc};
        block_partial<1>(v, part);
    }
};

template <typename V, typename V64, typename P, typename I, typename T, bool LR>
__global__ __launch_bounds__(kBlock) void k_persist(PersistSolve a) {
    __shared__ u32x4 lv[Chunks<double>::LDS];   // staging for the widest value type
    __shared__ u32x4 lc[Chunks<I>::LDS];
    __shared__ int64_t dict[kCodeDict];
    __shared__ unsigned s_gen0;
    const P *rp = static_cast<const P *>(a.rp);
    const I *ci = static_cast<const I *>(a.ci);
    const int64_t n = a.n;
    const int G = gridDim.x;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if constexpr (std::is_same_v<I, Code8>) {
        const int64_t *g = reinterpret_cast<const int64_t *>(ci) - kCodeDict;
        for (int i = threadIdx.x; i < kCodeDict; i += kBlock) dict[i] = g[i];
    }
    if (threadIdx.x == 0) s_gen0 = __hip_atomic_load(&a.bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    unsigned gen = s_gen0;
    auto sync = [&]() { return grid_sync(a.bar, gen, a.spin_ticks); };
    // one pass over this workgroup's tiles with values va (type W), gather gx
    // and row sums accumulated in the type of ctag
    auto tiles = [&](auto ctag, const auto *va, const auto &gx, auto &epi) {
        using W = std::remove_const_t<std::remove_pointer_t<decltype(va)>>;
        using C = decltype(ctag);
        if constexpr (std::is_same_v<I, Code8>)
            spmv_tiles_lds<W, P, I, C, LR>(n, a.nnz, rp, ci, va, gx, a.remap, a.nt, 1, epi, lv, lc, ColCoded{dict});
        else
            spmv_tiles_lds<W, P, I, C, LR>(n, a.nnz, rp, ci, va, gx, a.remap, a.nt, 1, epi, lv, lc, ColPlain{});
        epi.finish();
    };
    double *part_init = a.partials + static_cast<size_t>(SITE_INIT) * kSiteWidth * kMaxGrid;
    double *part_fcg = a.partials + static_cast<size_t>(SITE_FCG) * kSiteWidth * kMaxGrid;
    double *part_true = a.partials + static_cast<size_t>(SITE_TRUE) * kSiteWidth * kMaxGrid;
    const int64_t vstride = static_cast<int64_t>(G) * kBlock;
    const int64_t vfirst = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;

    // the fused steps k = 0, 1, ... on buffers f (x: the solution, FP64 x or
    // the inner correction d) until a decision stops them; returns the stop
    // reason and the completed iterations (0 with an error return of -1)
    auto steps = [&](const V *va, const FcgBufs<T> &f, T *x, double thresh, int64_t max_it, SolveState *st,
                     int64_t &done_out) -> int {
        for (int64_t k = 0;; ++k) {
            EpiStep<T> rw;
            rw.bind(f, x, k);
            const bool odd = (k & 1) != 0;
            rw.part = part_fcg + (odd ? static_cast<size_t>(4) * kMaxGrid : 0);
            if (k >= 1) {
                double tot[4];
                sum_partials<4>(part_fcg + (odd ? 0 : static_cast<size_t>(4) * kMaxGrid), G, tot);
                double al = 0.0, be = 0.0;
                const int stop = fcg::decide(tot, k - 1, thresh, max_it, al, be);
                if (lead && st) {
                    fcg::record(st, tot, k - 1);
                    if (stop == STOP_RUNNING) st->alpha = al;
                }
                if (stop != STOP_RUNNING) {
                    done_out = k - 1;
                    return stop;
                }
                rw.alpha = static_cast<T>(al);
                rw.beta = static_cast<T>(be);
            }
            tiles(T(0), va, rw.gather(), rw);   // the inner product accumulates in the vector type
            if (!sync()) return -1;
        }
    };

    if constexpr (std::is_same_v<T, double>) {
        // ---------------- FP64 CG
        const V *va = static_cast<const V *>(a.va);
        FcgBufs<double> f = a.f64;
        {
            fcg::EpiInit e{a.b, f.r[1], f.p[1], f.q[1], part_init, 0.0, 0.0};
            tiles(0.0, va, PlainGather<double, double>{a.x}, e);
        }
        if (!sync()) return;
        double t2[2];
        sum_partials<2>(part_init, G, t2);
        const double bn = sqrt(t2[1]), rho = t2[0], res = sqrt(rho);
        int stop = STOP_RUNNING, zero_x = 0;
        if (!isfinite(bn)) stop = STOP_NON_FINITE;
        else if (bn == 0.0) {
            stop = STOP_CONVERGED;
            zero_x = 1;
        } else if (!isfinite(rho)) stop = STOP_NON_FINITE;
        else if (res <= a.tau * bn) stop = STOP_CONVERGED;
        else if (a.max_iters <= 0) stop = STOP_MAX_ITERS;
        SolveState *S = a.st;
        if (lead) {
            S->x = a.x;
            S->hist = a.hist;
            S->hist_cap = a.hist_cap;
            S->max_iters = a.max_iters;
            S->base = 0;
            S->iter = 0;
            S->zero_x = zero_x;
            S->bnorm = bn;
            S->thresh = a.tau * bn;
            S->rho[0] = zero_x ? 0.0 : rho;
            S->resnorm = zero_x ? 0.0 : (isfinite(bn) ? res : bn);
            S->true_resnorm = zero_x ? 0.0 : __builtin_nan("");
            if (a.hist && a.hist_cap > 0) a.hist[0] = S->resnorm;
        }
        int64_t done = 0;
        if (stop == STOP_RUNNING) {
            stop = steps(va, f, a.x, a.tau * bn, a.max_iters, S, done);
            if (stop < 0) return;
        }
        if (lead) {
            S->iter = done;
            S->stop = stop;
        }
        if (zero_x) {
            for (int64_t i = vfirst; i < n; i += vstride) a.x[i] = 0.0;
            return;
        }
        if (!a.true_residual || stop == STOP_NON_FINITE) return;
        {
            EpiResid e{a.b, part_true, 0.0};
            tiles(0.0, va, PlainGather<double, double>{a.x}, e);
        }
        if (!sync()) return;
        double t1[1];
        sum_partials<1>(part_true, G, t1);
        if (lead) S->true_resnorm = sqrt(t1[0]);
    } else {
        // ---------------- FP32 inner CG inside FP64 refinement
        const V *va = static_cast<const V *>(a.va);
        const V64 *va64 = static_cast<const V64 *>(a.va64);
        FcgBufs<float> f = a.f32;
        int64_t inner_total = 0, outer = 0;
        double rn = 0.0, bn = 0.0;
        int stop = STOP_RUNNING;
        while (true) {
            {
                fcg::EpiIrResidual e{a.b, f.r[1], f.p[1], f.q[1], a.d32, part_init, 0.0, 0.0, 0.0};
                tiles(0.0, va64, PlainGather<double, double>{a.x}, e);   // FP64 accumulation
            }
            if (!sync()) return;
            double t3[3];
            sum_partials<3>(part_init, G, t3);
            rn = sqrt(t3[0]);
            bn = sqrt(t3[2]);
            const double r32n = sqrt(t3[1]);
            if (!isfinite(bn) || !isfinite(rn)) {
                stop = STOP_NON_FINITE;
                break;
            }
            if (bn == 0.0) {
                for (int64_t i = vfirst; i < n; i += vstride) a.x[i] = 0.0;
                rn = 0.0;
                stop = STOP_CONVERGED;
                break;
            }
            if (rn <= a.tau * bn) {
                stop = STOP_CONVERGED;
                break;
            }
            if (outer >= a.max_outer || inner_total >= a.max_iters) {
                stop = STOP_MAX_ITERS;
                break;
            }
            int64_t kin = 0;
            int in_stop = STOP_CONVERGED;   // r32 = 0: nothing to solve
            if (r32n != 0.0) {
                in_stop = steps(va, f, a.d32, a.tau_in * r32n, a.max_iters - inner_total, nullptr, kin);
                if (in_stop < 0) return;
            }
            inner_total += kin;
            if ((in_stop == STOP_BREAKDOWN || in_stop == STOP_NON_FINITE) && kin == 0) {
                stop = in_stop;
                break;
            }
            for (int64_t i = vfirst; i < n; i += vstride) a.x[i] += static_cast<double>(a.d32[i]);
            ++outer;
            if (!sync()) return;   // x complete before the next residual
        }
        if (lead) {
            a.res->inner = inner_total;
            a.res->outer = outer;
            a.res->rnorm = rn;
            a.res->bnorm = bn;
            a.res->stop = stop;
        }
    }
}

template <typename V, typename V64, typename P, typename I, typename T, bool LR>
const void *kernel_ptr() {
    return reinterpret_cast<const void *>(&k_persist<V, V64, P, I, T, LR>);
}

// The kernel for the solve's types (nullptr: no persistent kernel for them).
// outer: the refinement's matrix of a mixed solve (same index arrays as A),
// nullptr for an FP64 solve on A.  LR: with the long-row pass.
template <typename P, typename I, bool LR>
const void *kernel_values(const CsrDev &A, const CsrDev *outer) {
    if (!outer) return A.val_t == 0 ? kernel_ptr<double, double, P, I, double, LR>() : nullptr;
    if (A.val_t == 1 && outer->val_t == 0) return kernel_ptr<float, double, P, I, float, LR>();
    if (A.val_t == 1 && outer->val_t == 1) return kernel_ptr<float, float, P, I, float, LR>();
    if (A.val_t == 3 && outer->val_t == 0) return kernel_ptr<bf16s, double, P, I, float, LR>();
    if (A.val_t == 2 && outer->val_t == 0) return kernel_ptr<_Float16, double, P, I, float, LR>();
    return nullptr;
}

// Index combinations with a persistent kernel: int32 columns with int32 or
// int64 row pointers (with the long-row pass when the matrix has rows longer
// than kLongRow), and one-byte column codes with packed, int32 or int64 row
// pointers (coded matrices have no such rows).
const void *kernel_for(const CsrDev &A, const CsrDev *outer) {
    if (A.codes) {
        if (A.rowpack) return kernel_values<RowPack, Code8, false>(A, outer);
        if (A.ptr_t == 0) return kernel_values<int32_t, Code8, false>(A, outer);
        return kernel_values<int64_t, Code8, false>(A, outer);
    }
    if (A.idx_t != 0) return nullptr;
    const bool lr = A.max_row > kLongRow;
    if (A.ptr_t == 0)
        return lr ? kernel_values<int32_t, int32_t, true>(A, outer) : kernel_values<int32_t, int32_t, false>(A, outer);
    return lr ? kernel_values<int64_t, int32_t, true>(A, outer) : kernel_values<int64_t, int32_t, false>(A, outer);
}

}  // namespace

int persistent_blocks_per_cu(const CsrDev &A, const CsrDev *outer) {
    const void *k = kernel_for(A, outer);
    if (!k) return 0;
    int blocks = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, kBlock, 0);
    return (e == hipSuccess && blocks > 0) ? blocks : 0;
}

hipError_t launch_persistent(const CsrDev &A, const CsrDev *outer, PersistSolve a, int grid, hipStream_t s) {
    const void *k = kernel_for(A, outer);
    if (!k) return hipErrorInvalidValue;
    a.n = A.n_rows;
    a.nnz = A.nnz;
    a.rp = A.codes && A.rowpack ? A.rowpack : A.rp;
    a.ci = A.codes ? A.codes : A.ci;
    a.va = A.va;
    a.va64 = outer ? outer->va : A.va;
    void *args[] = {&a};
    return hipLaunchCooperativeKernel(k, dim3(grid), dim3(kBlock), args, 0, s);
}

}  // namespace spk
