// gfx950 kernels of the sparse Krylov hot path.
//
// SpMV (y = A x, the operator apply of Section 4.2) comes in two tilings that
// share one set of fused epilogues:
//   * LDS-staged row tiles: a workgroup owns 256 consecutive rows; it streams
//     the tile's values and column indices from HBM into LDS with fully
//     coalesced loads (one contiguous nnz range per tile), then each thread
//     reduces one row from LDS while gathering x.  Tiles whose nnz exceed the
//     LDS capacity fall back to direct loads.
//   * lanes-per-row vector kernel: 2^k lanes of a wave64 share a row.
// Workgroups walk tiles grid-stride; with xcd_remap each of the 8 XCDs walks
// one contiguous eighth of the tiles, so x-gathers of neighbouring rows share
// that XCD's L2.
//
// The CG solve (Section 6.2 benchmarks CG; the iteration is the textbook
// Hestenes-Stiefel one) runs as three launches per iteration:
//   spmv_pq : q = A p, p.q      -> alpha (or breakdown)
//   update  : x += alpha p, r -= alpha q, r.r -> stop test, beta
//   pupdate : p = r + beta p
// Every reduction is deterministic: each workgroup writes its FP64 partial,
// the last workgroup to arrive (agent-scope acq_rel counter) sums the
// partials in a fixed order and updates the device-resident SolveState.
// Kernels return at once when the state says the solve has stopped, so a
// chunk of iterations enqueued past convergence costs only empty launches.
#include "spk_internal.h"

#include <cmath>
#include <type_traits>

namespace spk {
namespace {

struct bf16s { uint16_t bits; };

__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ float widen(_Float16 v) { return static_cast<float>(v); }
__device__ __forceinline__ float widen(bf16s v) { return __uint_as_float(static_cast<unsigned>(v.bits) << 16); }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Tiles visited by this workgroup.
struct TileIter {
    int64_t t, end, stride;
    __device__ TileIter(int64_t T, int remap) {
        const int64_t G = gridDim.x, b = blockIdx.x;
        if (remap && G >= kNumXcd) {
            const int64_t xcd = b % kNumXcd, m = b / kNumXcd;
            const int64_t M = (G - xcd + kNumXcd - 1) / kNumXcd;   // workgroups on this XCD
            t = xcd * T / kNumXcd + m;
            end = (xcd + 1) * T / kNumXcd;
            stride = M;
        } else {
            t = b;
            end = T;
            stride = G;
        }
    }
};

// Deterministic grid reduction of NV doubles.  Every workgroup calls it once;
// the last to arrive runs last(tot) on thread 0 with the fixed-order totals.
template <int NV, class Last>
__device__ __forceinline__ void reduce_finish(double (&v)[NV], double *partials, unsigned *counter, Last last) {
    __shared__ double sh[NV][kBlock / 64];
    __shared__ int s_last;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double t = wave_sum(v[j]);
        if (lane == 0) sh[j][wid] = t;
    }
    __syncthreads();
    const unsigned G = gridDim.x;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double t = sh[j][0];
#pragma unroll
            for (int w = 1; w < kBlock / 64; ++w) t += sh[j][w];
            partials[j * kMaxGrid + blockIdx.x] = t;
        }
        const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == G - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double t = 0.0;
        for (unsigned b = threadIdx.x; b < G; b += kBlock) t += partials[j * kMaxGrid + b];
        t = wave_sum(t);
        if (lane == 0) sh[j][wid] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double t = sh[j][0];
#pragma unroll
            for (int w = 1; w < kBlock / 64; ++w) t += sh[j][w];
            tot[j] = t;
        }
        *counter = 0u;
        last(tot);
    }
}

// ------------------------------------------------------------------ epilogues
template <class X>
struct EpiPlain {
    X *y;
    __device__ bool skip() const { return false; }
    template <class C>
    __device__ void row(int64_t i, C s) { y[i] = static_cast<X>(s); }
    __device__ void finish() {}
};

// r = b - A x, p = r; reduces r.r and b.b, then sets up the solve state.
struct EpiInit {
    const double *b;
    double *r, *p, *x;
    SolveState *st;
    double *part;
    double tau;
    int64_t max_iters;
    double *hist;
    int64_t hist_cap;
    double rr, bb;
    __device__ bool skip() const { return false; }
    __device__ void row(int64_t i, double s) {
        const double bi = b[i];
        const double ri = bi - s;
        r[i] = ri;
        p[i] = ri;
        rr = fma(ri, ri, rr);
        bb = fma(bi, bi, bb);
    }
    __device__ void finish() {
        double v[2] = {rr, bb};
        SolveState *S = st;
        double *X = x, *H = hist;
        const int64_t hc = hist_cap, mi = max_iters;
        const double ta = tau;
        reduce_finish<2>(v, part, &S->counters[SITE_INIT], [=](const double *tot) {
            S->x = X;
            S->hist = H;
            S->hist_cap = hc;
            S->max_iters = mi;
            S->iter = 0;
            S->zero_x = 0;
            S->stop = STOP_RUNNING;
            S->alpha = 0.0;
            S->beta = 0.0;
            S->pq = 0.0;
            S->true_resnorm = __builtin_nan("");
            const double bn = sqrt(tot[1]);
            S->bnorm = bn;
            S->thresh = ta * bn;
            if (!isfinite(bn)) {
                S->stop = STOP_NON_FINITE;
                S->resnorm = bn;
            } else if (bn == 0.0) {
                S->zero_x = 1;
                S->stop = STOP_CONVERGED;
                S->resnorm = 0.0;
                S->true_resnorm = 0.0;
                S->rho = 0.0;
                if (H && hc > 0) H[0] = 0.0;
            } else {
                const double rho = tot[0];
                const double res = sqrt(rho);
                S->rho = rho;
                S->resnorm = res;
                if (H && hc > 0) H[0] = res;
                if (!isfinite(rho)) S->stop = STOP_NON_FINITE;
                else if (res <= ta * bn) S->stop = STOP_CONVERGED;
                else if (mi <= 0) S->stop = STOP_MAX_ITERS;
            }
        });
    }
};

// q = A p; reduces p.q and forms alpha = rho / p.q.
struct EpiPq {
    double *q;
    const double *p;
    SolveState *st;
    double *part;
    double acc;
    __device__ bool skip() const { return st->stop != STOP_RUNNING; }
    __device__ void row(int64_t i, double s) {
        q[i] = s;
        acc = fma(p[i], s, acc);
    }
    __device__ void finish() {
        double v[1] = {acc};
        SolveState *S = st;
        reduce_finish<1>(v, part, &S->counters[SITE_PQ], [=](const double *tot) {
            const double pq = tot[0];
            S->pq = pq;
            if (!isfinite(pq)) S->stop = STOP_NON_FINITE;
            else if (pq <= 0.0) S->stop = STOP_BREAKDOWN;
            else S->alpha = S->rho / pq;
        });
    }
};

// ||b - A x|| at exit.
struct EpiTrue {
    const double *b;
    SolveState *st;
    double *part;
    double acc;
    __device__ bool skip() const { return st->zero_x != 0 || st->stop == STOP_NON_FINITE; }
    __device__ void row(int64_t i, double s) {
        const double ri = b[i] - s;
        acc = fma(ri, ri, acc);
    }
    __device__ void finish() {
        double v[1] = {acc};
        SolveState *S = st;
        reduce_finish<1>(v, part, &S->counters[SITE_TRUE], [=](const double *tot) { S->true_resnorm = sqrt(tot[0]); });
    }
};

// ------------------------------------------------------------------ SpMV tilings
constexpr int kStreamCap = 2048;   // nnz staged in LDS per tile

template <typename V, typename P, typename I, typename X, typename C, class Epi>
__global__ __launch_bounds__(kBlock) void k_spmv_stream(int64_t n, const P *__restrict__ rp,
                                                        const I *__restrict__ ci, const V *__restrict__ va,
                                                        const X *__restrict__ x, int remap, Epi epi_in) {
    Epi epi = epi_in;
    if (epi.skip()) return;
    __shared__ V sv[kStreamCap];
    __shared__ I sc[kStreamCap];
    const int tid = threadIdx.x;
    const int64_t T = (n + kTileRows - 1) / kTileRows;
    for (TileIter it(T, remap); it.t < it.end; it.t += it.stride) {
        const int64_t r0 = it.t * kTileRows;
        const int64_t r1 = min(r0 + (int64_t)kTileRows, n);
        const int64_t row = r0 + tid;
        const int64_t s = static_cast<int64_t>(rp[r0]);
        const int64_t cnt = static_cast<int64_t>(rp[r1]) - s;
        int64_t a = 0, b = 0;
        if (row < r1) {
            a = static_cast<int64_t>(rp[row]) - s;
            b = static_cast<int64_t>(rp[row + 1]) - s;
        }
        if (cnt <= kStreamCap) {
            V tv[kStreamCap / kBlock];
            I tc[kStreamCap / kBlock];
#pragma unroll
            for (int u = 0; u < kStreamCap / kBlock; ++u) {
                const int64_t k = tid + u * kBlock;
                if (k < cnt) {
                    tv[u] = va[s + k];
                    tc[u] = ci[s + k];
                }
            }
#pragma unroll
            for (int u = 0; u < kStreamCap / kBlock; ++u) {
                const int64_t k = tid + u * kBlock;
                if (k < cnt) {
                    sv[k] = tv[u];
                    sc[k] = tc[u];
                }
            }
            __syncthreads();
            if (row < r1) {
                C sum = 0;
                for (int64_t k0 = a; k0 < b; k0 += 8) {
                    C av[8], xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int64_t k = k0 + u;
                        if (k < b) {
                            av[u] = static_cast<C>(widen(sv[k]));
                            xv[u] = static_cast<C>(x[sc[k]]);
                        } else {
                            av[u] = 0;
                            xv[u] = 0;
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) sum = fma(av[u], xv[u], sum);
                }
                epi.row(row, sum);
            }
            __syncthreads();
        } else if (row < r1) {
            C sum = 0;
            for (int64_t k = s + a; k < s + b; ++k) sum = fma(static_cast<C>(widen(va[k])), static_cast<C>(x[ci[k]]), sum);
            epi.row(row, sum);
        }
    }
    epi.finish();
}

template <typename V, typename P, typename I, typename X, typename C, class Epi>
__global__ __launch_bounds__(kBlock) void k_spmv_vector(int64_t n, const P *__restrict__ rp,
                                                        const I *__restrict__ ci, const V *__restrict__ va,
                                                        const X *__restrict__ x, int lanes_log2, int remap,
                                                        Epi epi_in) {
    Epi epi = epi_in;
    if (epi.skip()) return;
    const int L = 1 << lanes_log2;
    const int lane = threadIdx.x & (L - 1);
    const int group = threadIdx.x >> lanes_log2;
    const int groups = kBlock >> lanes_log2;
    const int64_t T = (n + kTileRows - 1) / kTileRows;
    for (TileIter it(T, remap); it.t < it.end; it.t += it.stride) {
        const int64_t r0 = it.t * kTileRows;
        const int64_t r1 = min(r0 + (int64_t)kTileRows, n);
        for (int pass = 0; pass < L; ++pass) {
            const int64_t row = r0 + static_cast<int64_t>(pass) * groups + group;
            C sum = 0;
            if (row < r1) {
                const int64_t a = static_cast<int64_t>(rp[row]), b = static_cast<int64_t>(rp[row + 1]);
                for (int64_t k = a + lane; k < b; k += L)
                    sum = fma(static_cast<C>(widen(va[k])), static_cast<C>(x[ci[k]]), sum);
            }
            for (int off = L >> 1; off >= 1; off >>= 1) sum += __shfl_xor(sum, off, 64);
            if (row < r1 && lane == 0) epi.row(row, sum);
        }
    }
    epi.finish();
}

template <class F>
hipError_t dispatch_idx(const CsrDev &A, F &&f) {
    if (A.ptr_t == 0) {
        if (A.idx_t == 0) return f(static_cast<const int32_t *>(A.rp), static_cast<const int32_t *>(A.ci));
        return f(static_cast<const int32_t *>(A.rp), static_cast<const int64_t *>(A.ci));
    }
    if (A.idx_t == 0) return f(static_cast<const int64_t *>(A.rp), static_cast<const int32_t *>(A.ci));
    return f(static_cast<const int64_t *>(A.rp), static_cast<const int64_t *>(A.ci));
}

template <class Ptr>
using pointee_t = std::remove_const_t<std::remove_pointer_t<Ptr>>;

template <typename V, typename X, typename C, class Epi>
hipError_t launch_family(const CsrDev &A, const SpmvTune &t, const X *x, const Epi &epi, hipStream_t s) {
    if (A.n_rows == 0) return hipSuccess;
    return dispatch_idx(A, [&](auto rp, auto ci) {
        using P = pointee_t<decltype(rp)>;
        using I = pointee_t<decltype(ci)>;
        const V *va = static_cast<const V *>(A.va);
        const dim3 grid(t.grid), block(kBlock);
        if (t.kind == 0)
            hipLaunchKernelGGL((k_spmv_stream<V, P, I, X, C, Epi>), grid, block, 0, s, A.n_rows, rp, ci, va, x,
                               t.xcd_remap, epi);
        else
            hipLaunchKernelGGL((k_spmv_vector<V, P, I, X, C, Epi>), grid, block, 0, s, A.n_rows, rp, ci, va, x,
                               t.lanes_log2, t.xcd_remap, epi);
        return hipGetLastError();
    });
}

// ------------------------------------------------------------------ vector kernels
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t n, const double *__restrict__ p,
                                                      double *__restrict__ r, const double *__restrict__ q,
                                                      SolveState *st, double *part) {
    if (st->stop != STOP_RUNNING) return;
    const double alpha = st->alpha;
    double *__restrict__ x = st->x;
    double acc = 0.0;
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    if ((reinterpret_cast<uintptr_t>(x) & 15) == 0) {
        const int64_t n2 = n >> 1;
        double2 *x2 = reinterpret_cast<double2 *>(x);
        double2 *r2 = reinterpret_cast<double2 *>(r);
        const double2 *p2 = reinterpret_cast<const double2 *>(p);
        const double2 *q2 = reinterpret_cast<const double2 *>(q);
        for (int64_t i = gid; i < n2; i += stride) {
            double2 xv = x2[i], rv = r2[i];
            const double2 pv = p2[i], qv = q2[i];
            xv.x = fma(alpha, pv.x, xv.x);
            xv.y = fma(alpha, pv.y, xv.y);
            rv.x = fma(-alpha, qv.x, rv.x);
            rv.y = fma(-alpha, qv.y, rv.y);
            x2[i] = xv;
            r2[i] = rv;
            acc = fma(rv.x, rv.x, acc);
            acc = fma(rv.y, rv.y, acc);
        }
        if ((n & 1) && gid == 0) {
            const int64_t i = n - 1;
            x[i] = fma(alpha, p[i], x[i]);
            const double ri = fma(-alpha, q[i], r[i]);
            r[i] = ri;
            acc = fma(ri, ri, acc);
        }
    } else {
        for (int64_t i = gid; i < n; i += stride) {
            x[i] = fma(alpha, p[i], x[i]);
            const double ri = fma(-alpha, q[i], r[i]);
            r[i] = ri;
            acc = fma(ri, ri, acc);
        }
    }
    double v[1] = {acc};
    reduce_finish<1>(v, part, &st->counters[SITE_RR], [=](const double *tot) {
        const double rho_new = tot[0];
        const int64_t k = st->iter + 1;
        st->iter = k;
        const double res = sqrt(rho_new);
        st->resnorm = res;
        if (st->hist && k < st->hist_cap) st->hist[k] = res;
        if (!isfinite(rho_new)) {
            st->stop = STOP_NON_FINITE;
        } else if (res <= st->thresh) {
            st->stop = STOP_CONVERGED;
        } else if (k >= st->max_iters) {
            st->stop = STOP_MAX_ITERS;
        } else {
            st->beta = rho_new / st->rho;
            st->rho = rho_new;
        }
    });
}

__global__ __launch_bounds__(kBlock) void k_cg_pupdate(int64_t n, const double *__restrict__ r,
                                                       double *__restrict__ p, SolveState *st) {
    if (st->stop != STOP_RUNNING) return;
    const double beta = st->beta;
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    const int64_t n2 = n >> 1;
    const double2 *r2 = reinterpret_cast<const double2 *>(r);
    double2 *p2 = reinterpret_cast<double2 *>(p);
    for (int64_t i = gid; i < n2; i += stride) {
        const double2 rv = r2[i];
        double2 pv = p2[i];
        pv.x = fma(beta, pv.x, rv.x);
        pv.y = fma(beta, pv.y, rv.y);
        p2[i] = pv;
    }
    if ((n & 1) && gid == 0) p[n - 1] = fma(beta, p[n - 1], r[n - 1]);
}

__global__ __launch_bounds__(kBlock) void k_zero_x(int64_t n, SolveState *st) {
    if (!st->zero_x) return;
    double *x = st->x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) x[i] = 0.0;
}

// ------------------------------------------------------------------ structure kernels
template <typename P, typename I>
__global__ __launch_bounds__(kBlock) void k_validate(int64_t n_rows, int64_t n_cols, int64_t nnz,
                                                     const P *__restrict__ rp, const I *__restrict__ ci,
                                                     unsigned *flags) {
    unsigned f = 0;
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    if (gid == 0) {
        if (rp[0] != 0) f |= VFLAG_BAD_FIRST;
        if (static_cast<int64_t>(rp[n_rows]) != nnz) f |= VFLAG_BAD_LAST;
    }
    for (int64_t i = gid; i < n_rows; i += stride)
        if (rp[i + 1] < rp[i]) f |= VFLAG_DECREASING;
    for (int64_t k = gid; k < nnz; k += stride) {
        const int64_t c = static_cast<int64_t>(ci[k]);
        if (c < 0 || c >= n_cols) f |= VFLAG_BAD_COLUMN;
    }
    if (f) atomicOr(flags, f);
}

template <typename P>
__global__ __launch_bounds__(kBlock) void k_partition(int64_t n, const P *__restrict__ rp, int64_t parts,
                                                      int64_t *split) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (j > parts) return;
    if (j == parts) {
        split[j] = n;
        return;
    }
    const int64_t nnz = static_cast<int64_t>(rp[n]);
    const int64_t q = nnz / parts, rm = nnz % parts;
    const int64_t target = j * q + (j * rm) / parts;   // floor(j * nnz / parts) without overflow
    int64_t lo = 0, hi = n;                            // first i in [0, n] with rp[i] >= target
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (static_cast<int64_t>(rp[mid]) < target) lo = mid + 1;
        else hi = mid;
    }
    split[j] = lo;
}

__global__ __launch_bounds__(kBlock) void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n16) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

int grid_for(int64_t n, int per_thread, int cap) {
    const int64_t want = (n + static_cast<int64_t>(kBlock) * per_thread - 1) / (static_cast<int64_t>(kBlock) * per_thread);
    return static_cast<int>(want < 1 ? 1 : (want > cap ? cap : want));
}

}  // namespace

// ==================================================================== launchers
hipError_t launch_validate(const CsrDev &A, unsigned *flags, hipStream_t s) {
    const int64_t work = A.n_rows > A.nnz ? A.n_rows : A.nnz;
    const int grid = grid_for(work, 8, kMaxGrid);
    return dispatch_idx(A, [&](auto rp, auto ci) {
        using P = pointee_t<decltype(rp)>;
        using I = pointee_t<decltype(ci)>;
        hipLaunchKernelGGL((k_validate<P, I>), dim3(grid), dim3(kBlock), 0, s, A.n_rows, A.n_cols, A.nnz, rp, ci, flags);
        return hipGetLastError();
    });
}

hipError_t launch_partition(const CsrDev &A, int64_t parts, int64_t *split, hipStream_t s) {
    const int64_t blocks = (parts + 1 + kBlock - 1) / kBlock;
    if (A.ptr_t == 0)
        hipLaunchKernelGGL((k_partition<int32_t>), dim3(blocks), dim3(kBlock), 0, s, A.n_rows,
                           static_cast<const int32_t *>(A.rp), parts, split);
    else
        hipLaunchKernelGGL((k_partition<int64_t>), dim3(blocks), dim3(kBlock), 0, s, A.n_rows,
                           static_cast<const int64_t *>(A.rp), parts, split);
    return hipGetLastError();
}

hipError_t launch_spmv(const CsrDev &A, const SpmvTune &t, const void *x, void *y, hipStream_t s) {
    switch (A.val_t) {
        case 0:
            return launch_family<double, double, double>(A, t, static_cast<const double *>(x),
                                                         EpiPlain<double>{static_cast<double *>(y)}, s);
        case 1:
            return launch_family<float, float, float>(A, t, static_cast<const float *>(x),
                                                      EpiPlain<float>{static_cast<float *>(y)}, s);
        case 2:
            return launch_family<_Float16, float, float>(A, t, static_cast<const float *>(x),
                                                         EpiPlain<float>{static_cast<float *>(y)}, s);
        case 3:
            return launch_family<bf16s, float, float>(A, t, static_cast<const float *>(x),
                                                      EpiPlain<float>{static_cast<float *>(y)}, s);
        default:
            return hipErrorInvalidValue;
    }
}

static double *site(double *partials, int k) { return partials + static_cast<size_t>(k) * kSiteWidth * kMaxGrid; }

hipError_t launch_cg_init(const CsrDev &A, const SpmvTune &t, const double *b, double *x, double *r, double *p,
                          SolveState *st, double *partials, double tau, int64_t max_iters, double *hist,
                          int64_t hist_cap, hipStream_t s) {
    EpiInit e{b, r, p, x, st, site(partials, SITE_INIT), tau, max_iters, hist, hist_cap, 0.0, 0.0};
    return launch_family<double, double, double>(A, t, x, e, s);
}

hipError_t launch_cg_spmv_pq(const CsrDev &A, const SpmvTune &t, const double *p, double *q, SolveState *st,
                             double *partials, hipStream_t s) {
    EpiPq e{q, p, st, site(partials, SITE_PQ), 0.0};
    return launch_family<double, double, double>(A, t, p, e, s);
}

hipError_t launch_cg_update(int64_t n, int grid, const double *p, double *r, const double *q, SolveState *st,
                            double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_update, dim3(grid), dim3(kBlock), 0, s, n, p, r, q, st, site(partials, SITE_RR));
    return hipGetLastError();
}

hipError_t launch_cg_pupdate(int64_t n, int grid, const double *r, double *p, SolveState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_pupdate, dim3(grid), dim3(kBlock), 0, s, n, r, p, st);
    return hipGetLastError();
}

hipError_t launch_cg_finalize(const CsrDev &A, const SpmvTune &t, const double *b, double *x_caller,
                              SolveState *st, double *partials, int true_residual, hipStream_t s) {
    (void)x_caller;
    hipLaunchKernelGGL(k_zero_x, dim3(grid_for(A.n_rows, 8, kMaxGrid)), dim3(kBlock), 0, s, A.n_rows, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !true_residual) return e;
    EpiTrue et{b, st, site(partials, SITE_TRUE), 0.0};
    return launch_family<double, double, double>(A, t, x_caller, et, s);
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(kBlock), 0, s, static_cast<const uint4 *>(src),
                       static_cast<uint4 *>(dst), static_cast<int64_t>(bytes / 16));
    return hipGetLastError();
}

int spmv_blocks_per_cu(const CsrDev &A, const SpmvTune &t) {
    int blocks = 0;
    hipError_t e = hipSuccess;
    auto q = [&](auto kern) { e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, kBlock, 0); };
    const bool i64 = A.idx_t != 0;
    if (A.val_t == 0) {
        if (t.kind == 0) {
            if (i64) q(k_spmv_stream<double, int64_t, int64_t, double, double, EpiPq>);
            else q(k_spmv_stream<double, int64_t, int32_t, double, double, EpiPq>);
        } else {
            if (i64) q(k_spmv_vector<double, int64_t, int64_t, double, double, EpiPq>);
            else q(k_spmv_vector<double, int64_t, int32_t, double, double, EpiPq>);
        }
    } else {
        if (t.kind == 0) q(k_spmv_stream<float, int64_t, int32_t, float, float, EpiPlain<float>>);
        else q(k_spmv_vector<float, int64_t, int32_t, float, float, EpiPlain<float>>);
    }
    if (e != hipSuccess || blocks < 1) blocks = 1;
    return blocks;
}

}  // namespace spk
