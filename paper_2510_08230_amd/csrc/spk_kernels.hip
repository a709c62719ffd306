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
// Hestenes-Stiefel one) runs as three launches per iteration k:
//   spmv_pq : q = A p_k, partials of p.q
//   update  : alpha = rho_k / p.q; x += alpha p, r -= alpha q; partials of r.r
//   pupdate : rho_{k+1} = r.r, stop test, beta; p = r + beta p
// Reductions need no atomics and no cache-flushing fences: each workgroup of
// the producing launch stores one FP64 partial, and every workgroup of the
// consuming launch re-sums all partials in the same fixed order, so all take
// identical decisions (launch boundaries make the partials visible across
// XCDs).  Per-iteration scalars live in a 4-slot ring indexed by the absolute
// iteration (chunk base + index within the chunk), so no launch reads a
// location that it writes.  Kernels return at once when the stop flag is
// set, so iterations enqueued past convergence cost only empty launches.
#include "spk_fcg.h"
#include "spk_launch.h"
#include "spk_spmv.h"

#include <climits>
#include <cmath>
#include <type_traits>

namespace spk {
namespace {

using namespace dev;
using namespace tile;

// ------------------------------------------------------------------ epilogues
template <class X>
struct EpiPlain {
    X *y;
    __device__ bool skip() const { return false; }
    template <class C>
    __device__ void row(int64_t i, C s) { y[i] = static_cast<X>(s); }
    __device__ void finish() {}
};

// r = b - A x, p = r; partials of r.r and b.b.
struct EpiInit {
    const double *b;
    double *r, *p;
    double *part;
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
        block_partial<2>(v, part);
    }
};

// q = A p (stored in T); partials of p.q accumulated in FP64 from the stored values.
template <typename T>
struct EpiPq {
    static constexpr bool kHotLoop = true;   // the CG loop's product (register budget of its kernel)
    T *q;
    const T *p;
    const SolveState *st;
    double *part;
    double acc;
    __device__ bool skip() const { return st->stop != STOP_RUNNING; }
    __device__ T pre(int64_t i) const { return p[i]; }
    template <class C>
    __device__ void row(int64_t i, C s, T pi) {
        const T qi = static_cast<T>(s);
        q[i] = qi;
        acc = fma(static_cast<double>(pi), static_cast<double>(qi), acc);
    }
    template <class C>
    __device__ void row(int64_t i, C s) { row(i, s, p[i]); }
    __device__ void finish() {
        double v[1] = {acc};
        block_partial<1>(v, part);
    }
};

// Refinement step of the mixed-precision solve: r = b - A x in FP64, then the
// inner right-hand side r32 = p32 = fl32(r) and d32 = 0; partials of ||r||^2
// (FP64), ||r32||^2 (FP64 sums of the rounded values) and ||b||^2.
struct EpiIrResidual {
    const double *b;
    float *r32, *p32, *d32;
    double *part;
    double rr, rr32, bb;
    __device__ bool skip() const { return false; }
    __device__ void row(int64_t i, double s) {
        const double bi = b[i];
        const double ri = bi - s;
        const float ri32 = static_cast<float>(ri);
        r32[i] = ri32;
        p32[i] = ri32;
        d32[i] = 0.0f;
        rr = fma(ri, ri, rr);
        rr32 = fma(static_cast<double>(ri32), static_cast<double>(ri32), rr32);
        bb = fma(bi, bi, bb);
    }
    __device__ void finish() {
        double v[3] = {rr, rr32, bb};
        block_partial<3>(v, part);
    }
};

// Partials of ||b - A x||^2 at exit.
struct EpiTrue {
    const double *b;
    const SolveState *st;
    double *part;
    double acc;
    __device__ bool skip() const { return st->zero_x != 0 || st->stop == STOP_NON_FINITE; }
    __device__ void row(int64_t i, double s) {
        const double ri = b[i] - s;
        acc = fma(ri, ri, acc);
    }
    __device__ void finish() {
        double v[1] = {acc};
        block_partial<1>(v, part);
    }
};

// ------------------------------------------------------------------ fused CG step
// One launch per CG iteration (the step and its decisions are described in
// spk_fcg.h).  The prologue runs in skip(): every workgroup sums the partials
// the previous step left and takes the same stop decision.
template <typename T>
struct EpiFcg : fcg::Rows<T> {
    FcgBufs<T> buf;
    SolveState *st;
    double *part;   // two sets of 4 slabs of kMaxGrid: set s at part + 4 s kMaxGrid
    int G;          // workgroups of every step (partials per slab)
    int j;          // step index within the chunk
    int w;
    __device__ bool skip() {
        // one read of the flag per workgroup: workgroup 0 may set it during
        // this launch, and all waves of a workgroup must take the same branch
        __shared__ int s_stop;
        if (threadIdx.x == 0) s_stop = st->stop;
        __syncthreads();
        if (s_stop != STOP_RUNNING) return true;
        const int64_t k = st->base + j;
        w = static_cast<int>(k & 1);
        this->bind(buf, static_cast<T *>(st->x), k);
        if (k == 0) return false;
        double tot[4];
        sum_partials<4>(part + (w ? 0 : static_cast<size_t>(4) * kMaxGrid), G, tot);
        const int64_t done = k - 1;   // x holds x_{k-1}
        double a = 0.0, b = 0.0;
        const int stop = fcg::decide(tot, done, st->thresh, st->max_iters, a, b);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            fcg::record(st, tot, done);
            if (stop == STOP_RUNNING) st->alpha = a;
            else st->stop = stop;   // every workgroup took the same decision
        }
        if (stop != STOP_RUNNING) return true;
        this->alpha = static_cast<T>(a);
        this->beta = static_cast<T>(b);
        return false;
    }
    __device__ void finish() { block_partial<4>(this->acc, part + (w ? static_cast<size_t>(4) * kMaxGrid : 0)); }
};

// ------------------------------------------------------------------ CG scalar + vector kernels
// One workgroup: finish the initial residual (||b||, rho_0, first stop test).
__global__ __launch_bounds__(kBlock) void k_init_finish(SolveState *st, const double *part, int G, double tau,
                                                        int64_t max_iters, double *x, double *hist, int64_t hist_cap) {
    double tot[2];
    sum_partials<2>(part, G, tot);
    if (threadIdx.x != 0) return;
    st->x = x;
    st->hist = hist;
    st->hist_cap = hist_cap;
    st->max_iters = max_iters;
    st->base = 0;
    st->iter = 0;
    st->zero_x = 0;
    st->stop = STOP_RUNNING;
    st->alpha = 0.0;
    st->pq = 0.0;
    st->true_resnorm = __builtin_nan("");
    const double bn = sqrt(tot[1]);
    st->bnorm = bn;
    st->thresh = tau * bn;
    if (!isfinite(bn)) {
        st->stop = STOP_NON_FINITE;
        st->resnorm = bn;
    } else if (bn == 0.0) {
        st->zero_x = 1;
        st->stop = STOP_CONVERGED;
        st->resnorm = 0.0;
        st->true_resnorm = 0.0;
        st->rho[0] = 0.0;
        if (hist && hist_cap > 0) hist[0] = 0.0;
    } else {
        const double rho = tot[0];
        const double res = sqrt(rho);
        st->rho[0] = rho;
        st->resnorm = res;
        if (hist && hist_cap > 0) hist[0] = res;
        if (!isfinite(rho)) st->stop = STOP_NON_FINITE;
        else if (res <= tau * bn) st->stop = STOP_CONVERGED;
        else if (max_iters <= 0) st->stop = STOP_MAX_ITERS;
    }
}


// r -= alpha q with alpha = rho_k / (p . q) (FP64 scalar, applied in T);
// partials of r.r accumulated in FP64.  x += alpha p is left to the p-update
// kernel, which reads p anyway.  j: index of this iteration within the chunk.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t n, T *__restrict__ r, const T *__restrict__ q,
                                                      SolveState *st, const double *part_pq, int G_pq,
                                                      double *part_rr, int j) {
    if (st->stop != STOP_RUNNING) return;
    const int64_t k = st->base + j;
    double tot[1];
    sum_partials<1>(part_pq, G_pq, tot);
    const double pq = tot[0];
    if (!isfinite(pq) || pq <= 0.0) {   // every workgroup sees the same pq and stops alike
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->pq = pq;
            st->stop = isfinite(pq) ? STOP_BREAKDOWN : STOP_NON_FINITE;
        }
        return;
    }
    const double alpha_d = st->rho[k & 3] / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->pq = pq;
        st->alpha = alpha_d;
    }
    const T alpha = static_cast<T>(alpha_d);
    double acc = 0.0;
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    constexpr int W = Vec16<T>::W;
    using VT = typename Vec16<T>::type;
    const int64_t nv = n / W;
    VT *rv_ = reinterpret_cast<VT *>(r);
    const VT *qv_ = reinterpret_cast<const VT *>(q);
    for (int64_t i = gid; i < nv; i += stride) {
        VT rv = rv_[i];
        const VT qv = qv_[i];
#pragma unroll
        for (int c = 0; c < W; ++c) {
            rv[c] = fma(-alpha, qv[c], rv[c]);
            acc = fma(static_cast<double>(rv[c]), static_cast<double>(rv[c]), acc);
        }
        rv_[i] = rv;
    }
    for (int64_t i = nv * W + gid; i < n; i += stride) {
        const T ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        acc = fma(static_cast<double>(ri), static_cast<double>(ri), acc);
    }
    double v[1] = {acc};
    block_partial<1>(v, part_rr);
}

// End of iteration k: x += alpha_k p_k (deferred from the update), then the
// stop test on rho_{k+1} = r.r (partials of the update kernel), beta =
// rho_{k+1} / rho_k and, unless stopping, p = r + beta p.  One pass over
// x, p and r.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_pupdate(int64_t n, const T *__restrict__ r, T *__restrict__ p,
                                                       SolveState *st, const double *part_rr, int G_rr, int j) {
    if (st->stop != STOP_RUNNING) return;   // breakdown in the update: x keeps x_k
    const int64_t k = st->base + j;
    double tot[1];
    sum_partials<1>(part_rr, G_rr, tot);
    const double rho_new = tot[0];
    const int64_t k1 = k + 1;
    const double res = sqrt(rho_new);
    int stop = STOP_RUNNING;
    if (!isfinite(rho_new)) stop = STOP_NON_FINITE;
    else if (res <= st->thresh) stop = STOP_CONVERGED;
    else if (k1 >= st->max_iters) stop = STOP_MAX_ITERS;
    const double beta_d = rho_new / st->rho[k & 3];
    const T alpha = static_cast<T>(st->alpha);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->iter = k1;
        st->resnorm = res;
        st->rho[k1 & 3] = rho_new;
        if (st->hist && k1 < st->hist_cap) st->hist[k1] = res;
        if (stop != STOP_RUNNING) st->stop = stop;
    }
    const T beta = static_cast<T>(beta_d);
    T *__restrict__ x = static_cast<T *>(st->x);
    const bool more = stop == STOP_RUNNING;
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    constexpr int W = Vec16<T>::W;
    using VT = typename Vec16<T>::type;
    int64_t done = 0;
    if ((reinterpret_cast<uintptr_t>(x) & 15) == 0) {
        const int64_t nv = n / W;
        VT *xv_ = reinterpret_cast<VT *>(x);
        VT *pv_ = reinterpret_cast<VT *>(p);
        const VT *rv_ = reinterpret_cast<const VT *>(r);
        if (more) {
            for (int64_t i = gid; i < nv; i += stride) {
                VT xv = xv_[i], pv = pv_[i];
                const VT rv = rv_[i];
#pragma unroll
                for (int c = 0; c < W; ++c) {
                    xv[c] = fma(alpha, pv[c], xv[c]);
                    pv[c] = fma(beta, pv[c], rv[c]);
                }
                xv_[i] = xv;
                pv_[i] = pv;
            }
        } else {
            for (int64_t i = gid; i < nv; i += stride) {
                VT xv = xv_[i];
                const VT pv = pv_[i];
#pragma unroll
                for (int c = 0; c < W; ++c) xv[c] = fma(alpha, pv[c], xv[c]);
                xv_[i] = xv;
            }
        }
        done = nv * W;
    }
    for (int64_t i = done + gid; i < n; i += stride) {
        const T pi = p[i];
        x[i] = fma(alpha, pi, x[i]);
        if (more) p[i] = fma(beta, pi, r[i]);
    }
}

// Refinement: finish the outer residual (||r64||, the outer stop test) and
// set up the inner CG on A32 d = r32 from d = 0 (rho_0 = ||r32||^2).
// out[0] = ||r64||, out[1] = ||r32|| (read by the host after the launch).
__global__ __launch_bounds__(kBlock) void k_ir_finish(SolveState *in, const double *part, int G, double tau_in,
                                                      int64_t max_inner, float *d32, double *out) {
    double tot[3];
    sum_partials<3>(part, G, tot);
    if (threadIdx.x != 0) return;
    out[0] = sqrt(tot[0]);
    out[2] = sqrt(tot[2]);
    const double r32 = sqrt(tot[1]);
    out[1] = r32;
    in->x = d32;
    in->hist = nullptr;
    in->hist_cap = 0;
    in->max_iters = max_inner;
    in->base = 0;
    in->iter = 0;
    in->zero_x = 0;
    in->alpha = 0.0;
    in->pq = 0.0;
    in->bnorm = r32;
    in->thresh = tau_in * r32;
    in->rho[0] = tot[1];
    in->resnorm = r32;
    in->stop = STOP_RUNNING;
    if (!isfinite(tot[0]) || !isfinite(tot[1])) in->stop = STOP_NON_FINITE;
    else if (r32 == 0.0) in->stop = STOP_CONVERGED;
    else if (max_inner <= 0) in->stop = STOP_MAX_ITERS;
}

// x64 += d32 after an inner solve.
__global__ __launch_bounds__(kBlock) void k_ir_correct(int64_t n, double *__restrict__ x, const float *__restrict__ d) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride)
        x[i] += static_cast<double>(d[i]);
}

// Round FP64 matrix values to the inner-solve storage type.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_round_values(int64_t nnz, const double *__restrict__ src, V *__restrict__ dst);

template <>
__global__ __launch_bounds__(kBlock) void k_round_values<float>(int64_t nnz, const double *__restrict__ src,
                                                               float *__restrict__ dst) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < nnz; i += stride)
        dst[i] = static_cast<float>(src[i]);
}

// FP64 -> bfloat16, rounded once to nearest even (NaN kept quiet).  The
// FP64 value is first narrowed to FP32 rounding to odd (truncate, then set
// the last bit if anything was dropped), which keeps the information the
// second rounding needs: FP32 carries 24 bits, more than bfloat16's 8 + 2,
// so nearest-even from the odd-rounded FP32 equals nearest-even from FP64
// (Boldo & Melquiond, round-to-odd).
__device__ __forceinline__ uint16_t to_bf16_rne(double v) {
    const float t = __double2float_rz(v);
    unsigned u = __float_as_uint(t);
    if ((u & 0x7f800000u) == 0x7f800000u) {   // Inf or NaN (truncation cannot overflow to Inf)
        if (u & 0x7fffffu) return static_cast<uint16_t>((u >> 16) | 0x40u);
        return static_cast<uint16_t>(u >> 16);
    }
    if (static_cast<double>(t) != v) u |= 1u;   // sticky: round to odd
    const unsigned rounding = 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>((u + rounding) >> 16);
}

template <>
__global__ __launch_bounds__(kBlock) void k_round_values<bf16s>(int64_t nnz, const double *__restrict__ src,
                                                               bf16s *__restrict__ dst) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < nnz; i += stride)
        dst[i].bits = to_bf16_rne(src[i]);
}

// FP64 -> binary16: the compiler's conversion rounds once to nearest even
// (subnormal halves and overflow to Inf included).
template <>
__global__ __launch_bounds__(kBlock) void k_round_values<_Float16>(int64_t nnz, const double *__restrict__ src,
                                                                  _Float16 *__restrict__ dst) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < nnz; i += stride)
        dst[i] = static_cast<_Float16>(src[i]);
}

// Advance the chunk base after `count` iterations (one thread).
__global__ void k_chunk_end(SolveState *st, int count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) st->base += count;
}

__global__ __launch_bounds__(kBlock) void k_true_finish(SolveState *st, const double *part, int G) {
    if (st->zero_x != 0 || st->stop == STOP_NON_FINITE) return;
    double tot[1];
    sum_partials<1>(part, G, tot);
    if (threadIdx.x == 0) st->true_resnorm = sqrt(tot[0]);
}

__global__ __launch_bounds__(kBlock) void k_zero_x(int64_t n, const SolveState *st) {
    if (!st->zero_x) return;
    double *x = static_cast<double *>(st->x);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) x[i] = 0.0;
}

// ------------------------------------------------------------------ structure kernels
constexpr int kValidateUnroll = 4;

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
    // Both walks take kValidateUnroll strides per round with every load of
    // the round issued before the first check, so each lane keeps that many
    // loads in flight (one at a time left the pass latency-bound).
    unsigned longest = 0;   // longest row (entries, clamped to 2^32 - 1), for the long-row path of the SpMV
    for (int64_t i0 = gid; i0 < n_rows; i0 += kValidateUnroll * stride) {
        int64_t lo[kValidateUnroll], hi[kValidateUnroll];
#pragma unroll
        for (int u = 0; u < kValidateUnroll; ++u) {
            const int64_t i = i0 + u * stride < n_rows ? i0 + u * stride : n_rows - 1;
            lo[u] = static_cast<int64_t>(rp[i]);
            hi[u] = static_cast<int64_t>(rp[i + 1]);
        }
#pragma unroll
        for (int u = 0; u < kValidateUnroll; ++u) {
            if (i0 + u * stride >= n_rows) continue;
            const int64_t len = hi[u] - lo[u];
            if (len < 0) f |= VFLAG_DECREASING;
            else longest = max(longest, len > 0xffffffffll ? 0xffffffffu : static_cast<unsigned>(len));
        }
    }
    // one atomic per workgroup at most: every wave's maximum goes through LDS,
    // and a maximum the flag word already holds (it only grows) is not sent
    // (same-address atomics from every wave serialised the pass)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) longest = max(longest, static_cast<unsigned>(__shfl_xor(longest, off, 64)));
    __shared__ unsigned wave_longest[kBlock / 64];
    if ((threadIdx.x & 63) == 0) wave_longest[threadIdx.x >> 6] = longest;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned m = wave_longest[0];
#pragma unroll
        for (int w = 1; w < kBlock / 64; ++w) m = max(m, wave_longest[w]);
        if (m > __hip_atomic_load(flags + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(flags + 1, m);
    }
    // column indices: 16-byte loads when aligned, element loads for the tail
    constexpr int EPC = 16 / sizeof(I);
    int64_t done = 0;
    if ((reinterpret_cast<uintptr_t>(ci) & 15) == 0) {
        const int64_t nch = nnz / EPC;
        const u32x4 *c16 = reinterpret_cast<const u32x4 *>(ci);
        for (int64_t g0 = gid; g0 < nch; g0 += kValidateUnroll * stride) {
            // chunks past the end re-read the last one (checked, not used)
            u32x4 v[kValidateUnroll];
#pragma unroll
            for (int u = 0; u < kValidateUnroll; ++u) {
                const int64_t g = g0 + u * stride;
                v[u] = c16[g < nch ? g : nch - 1];
            }
#pragma unroll
            for (int u = 0; u < kValidateUnroll; ++u) {
                if (g0 + u * stride >= nch) continue;
                I e[EPC];
                __builtin_memcpy(e, &v[u], 16);
#pragma unroll
                for (int j = 0; j < EPC; ++j) {
                    const int64_t c = static_cast<int64_t>(e[j]);
                    if (c < 0 || c >= n_cols) f |= VFLAG_BAD_COLUMN;
                }
            }
        }
        done = nch * EPC;
    }
    for (int64_t k = done + gid; k < nnz; k += stride) {
        const int64_t c = static_cast<int64_t>(ci[k]);
        if (c < 0 || c >= n_cols) f |= VFLAG_BAD_COLUMN;
    }
    if (f) atomicOr(flags, f);
}

// ------------------------------------------------------------------ column codes
// Plan-time derivation of the one-byte column codes that the LDS-tile SpMV can
// stream in place of column indices: index compression by offset from the
// row, for patterns with few distinct offsets c - i (stencils, banded
// matrices).  Random patterns overflow the table and keep their indices.
//   k_code_collect: each workgroup gathers the distinct offsets of its tiles
//     (all tiles, or every step-th tile and the last one) in an LDS hash
//     set, then merges them into the global open-addressing table; more than
//     kCodeDict distinct offsets sets the overflow word.
//   k_code_table: one workgroup ranks the table's offsets into an ascending
//     kCodeDict-entry table (unused entries 0), unless the collection
//     overflowed.
//   k_code_encode: every entry's offset is looked up (an LDS hash map built
//     from that table) and its position stored as one byte; an offset missing from the
//     table (possible after a sampled collection) sets the error word, and
//     the plan collects again over every tile, or keeps the plain indices.
// The three launch back to back; the host reads the words once at the end.
// words[0] = distinct offsets, words[1] = overflow (1) / missing code (2).
constexpr int kCodeLdsSlots = 512;
constexpr long long kCodeEmpty = LLONG_MIN;   // below every offset -(n - 1) .. n - 1

__device__ __forceinline__ unsigned code_hash(long long d, int bits) {
    return static_cast<unsigned>((static_cast<unsigned long long>(d) * 0x9E3779B97F4A7C15ull) >> (64 - bits));
}

__global__ __launch_bounds__(kBlock) void k_code_clear(long long *table, unsigned *words) {
    for (int i = threadIdx.x; i < kCodeSlots; i += kBlock) table[i] = kCodeEmpty;
    if (threadIdx.x < 4) words[threadIdx.x] = 0;
}

// Inserts d into an open-addressing set of 2^bits slots; returns 1 if this
// call placed it, 0 if it was present, -1 if every slot holds another value.
__device__ __forceinline__ int code_insert(long long *set, int bits, long long d) {
    const unsigned mask = (1u << bits) - 1u;
    unsigned h = code_hash(d, bits);
    for (unsigned probe = 0; probe <= mask; ++probe, h = (h + 1u) & mask) {
        long long v = set[h];
        if (v == d) return 0;
        if (v == kCodeEmpty) {
            v = static_cast<long long>(atomicCAS(reinterpret_cast<unsigned long long *>(set + h),
                                                 static_cast<unsigned long long>(kCodeEmpty),
                                                 static_cast<unsigned long long>(d)));
            if (v == kCodeEmpty) return 1;
            if (v == d) return 0;
        }
    }
    return -1;
}

// The entries of the 256-row tile at row r0, for the code kernels.
// CodeRows::load() reads the tile's row pointers (no LDS, no barrier: a walk
// issues it for its next tile before it works on the current one).
// CodeTile::cols() then, when the tile's entries fit the LDS row map (the
// usual case), issues the loads of entries s + threadIdx.x + j * kBlock
// (j < kCodeBatch; invalid past e), maps each entry to its row while they
// are in flight, and gives this thread those entries' offsets; otherwise
// mapped is false and each thread walks its own row [a, b).  Every thread
// of the workgroup must call cols() and done().  (Keeping the next tile's
// indices in flight as well cost a wave per SIMD and was slower.)
constexpr int kCodeBatch = kStreamCap / kBlock;

// The row pointers stay in their stored type until cols() (a widening right
// after the load would wait for it there).
template <typename P>
struct CodeRows {
    P s, e, a, b;
    int64_t r0;
    bool has;   // this thread's row is in the tile (else cols() clears a and b)
    __device__ __forceinline__ void load(int64_t n_rows, const P *__restrict__ rp, int64_t tile_r0) {
        r0 = tile_r0;
        const int64_t r1 = r0 + kTileRows < n_rows ? r0 + kTileRows : n_rows;
        s = rp[r0];
        e = rp[r1];
        const int64_t row = r0 + threadIdx.x;
        has = row < r1;
        const int64_t rr = has ? row : r1 - 1;   // unconditional loads (see cols())
        a = rp[rr];
        b = rp[rr + 1];
    }
};

template <typename P, typename I>
struct CodeTile {
    int64_t s, e, a, b, row, r0;
    bool mapped;
    int64_t d[kCodeBatch];
    __device__ __forceinline__ void cols(const CodeRows<P> &r, const I *__restrict__ ci, unsigned short *row_of) {
        r0 = r.r0;
        row = r0 + threadIdx.x;
        s = static_cast<int64_t>(r.s);
        e = static_cast<int64_t>(r.e);
        a = r.has ? static_cast<int64_t>(r.a) : 0;
        b = r.has ? static_cast<int64_t>(r.b) : 0;
        mapped = e - s <= kStreamCap;   // uniform
        if (!mapped) return;
        // every lane loads (entries past e re-read the tile's last one and
        // are not used): a load under a branch is waited for at the join
        I c[kCodeBatch];
        const int64_t last = e > s ? e - 1 : s;
        if (e > s) {   // uniform
#pragma unroll
            for (int j = 0; j < kCodeBatch; ++j) {
                const int64_t k = s + threadIdx.x + j * kBlock;
                c[j] = ci[k < last ? k : last];
            }
        }
        for (int64_t k = a; k < b; ++k) row_of[k - s] = static_cast<unsigned short>(threadIdx.x);
        lds_barrier();
#pragma unroll
        for (int j = 0; j < kCodeBatch; ++j) {
            const int64_t k = s + threadIdx.x + j * kBlock;
            d[j] = k < e ? static_cast<int64_t>(c[j]) - (r0 + row_of[k - s]) : 0;
        }
    }
    __device__ __forceinline__ bool valid(int j) const { return s + threadIdx.x + j * kBlock < e; }
    __device__ __forceinline__ int64_t entry(int j) const { return s + threadIdx.x + j * kBlock; }
    __device__ __forceinline__ void done() const {
        if (mapped) lds_barrier();   // row map free for the next tile
    }
};

// Tiles of the collection: every tile (step 1), or every step-th tile and the
// last one (a sample; the encode pass then proves the table complete).
__device__ __forceinline__ int64_t code_tiles(int64_t T, int step) { return (T + step - 1) / step + (step > 1); }
__device__ __forceinline__ int64_t code_tile(int64_t u, int64_t T, int step) {
    const int64_t t = u * step;
    return t < T ? t : T - 1;
}

template <typename P, typename I>
__global__ __launch_bounds__(kBlock) void k_code_collect(int64_t n_rows, const P *__restrict__ rp,
                                                         const I *__restrict__ ci, int step, long long *table,
                                                         unsigned *words) {
    __shared__ long long set[kCodeLdsSlots];
    __shared__ unsigned short row_of[kStreamCap];
    __shared__ unsigned used, over;
    for (int i = threadIdx.x; i < kCodeLdsSlots; i += kBlock) set[i] = kCodeEmpty;
    if (threadIdx.x == 0) used = over = 0;
    __syncthreads();
    const int64_t T = (n_rows + kTileRows - 1) / kTileRows;
    const int64_t U = code_tiles(T, step);
    auto add = [&](long long d) {
        const int r = code_insert(set, 9, d);
        if (r < 0 || (r > 0 && atomicAdd(&used, 1u) >= static_cast<unsigned>(kCodeDict))) over = 1;
    };
    CodeRows<P> nx;   // the next tile's row pointers, in flight while this one is worked on
    if (blockIdx.x < U) nx.load(n_rows, rp, code_tile(blockIdx.x, T, step) * kTileRows);
    for (int64_t u = blockIdx.x; u < U; u += gridDim.x) {
        CodeTile<P, I> t;
        t.cols(nx, ci, row_of);
        if (u + gridDim.x < U) nx.load(n_rows, rp, code_tile(u + gridDim.x, T, step) * kTileRows);
        if (t.mapped) {
#pragma unroll
            for (int j = 0; j < kCodeBatch; ++j)
                if (t.valid(j) && !over) add(t.d[j]);
        } else {
            for (int64_t k = t.a; k < t.b && !over; ++k) add(static_cast<long long>(ci[k]) - t.row);
        }
        t.done();
        lds_barrier();
        if (threadIdx.x == 0 && words[1]) over = 1;   // another workgroup already overflowed
        lds_barrier();
        if (over) break;                               // uniform: read after the barrier
    }
    if (over) {
        if (threadIdx.x == 0) atomicOr(&words[1], 1u);
        return;
    }
    for (int i = threadIdx.x; i < kCodeLdsSlots; i += kBlock) {
        const long long d = set[i];
        if (d == kCodeEmpty) continue;
        const int r = code_insert(table, 10, d);
        if (r < 0 || (r > 0 && atomicAdd(&words[0], 1u) >= static_cast<unsigned>(kCodeDict))) atomicOr(&words[1], 1u);
    }
}

__global__ __launch_bounds__(kBlock) void k_code_table(const long long *__restrict__ table,
                                                       const unsigned *__restrict__ words, int64_t *dict) {
    __shared__ long long t[kCodeDict];
    __shared__ long long out[kCodeDict];
    __shared__ unsigned cnt;
    if (words[1] != 0 || words[0] > static_cast<unsigned>(kCodeDict)) return;   // no codes: uniform
    if (threadIdx.x == 0) cnt = 0;
    for (int i = threadIdx.x; i < kCodeDict; i += kBlock) out[i] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < kCodeSlots; i += kBlock) {   // compact (at most kCodeDict entries)
        const long long d = table[i];
        if (d == kCodeEmpty) continue;
        const unsigned at = atomicAdd(&cnt, 1u);
        if (at < static_cast<unsigned>(kCodeDict)) t[at] = d;
    }
    __syncthreads();
    const int m = cnt < static_cast<unsigned>(kCodeDict) ? static_cast<int>(cnt) : kCodeDict;
    for (int i = threadIdx.x; i < m; i += kBlock) {
        int rank = 0;
        for (int j = 0; j < m; ++j) rank += t[j] < t[i] ? 1 : 0;
        out[rank] = t[i];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kCodeDict; i += kBlock) dict[i] = out[i];
}

// Code of offset d from the LDS hash map (keys / codes) the encode pass
// builds from the sorted table, or -1 when d is not in it.  One probe in the
// usual case (a binary search over the table took five times longer).
__device__ __forceinline__ int code_lookup(const long long *key, const unsigned char *code, long long d) {
    const unsigned mask = kCodeLdsSlots - 1u;
    unsigned h = code_hash(d, 9);
    for (unsigned probe = 0; probe <= mask; ++probe, h = (h + 1u) & mask) {
        const long long v = key[h];
        if (v == d) return code[h];
        if (v == kCodeEmpty) return -1;
    }
    return -1;
}

template <typename P, typename I>
__global__ __launch_bounds__(kBlock) void k_code_encode(int64_t n_rows, const P *__restrict__ rp,
                                                        const I *__restrict__ ci, const int64_t *__restrict__ dict,
                                                        uint8_t *__restrict__ codes, unsigned *words) {
    __shared__ long long key[kCodeLdsSlots];
    __shared__ unsigned char code[kCodeLdsSlots];
    __shared__ unsigned short row_of[kStreamCap];
    const unsigned nd = words[0];
    if (words[1] != 0 || nd < 1 || nd > static_cast<unsigned>(kCodeDict)) return;   // no codes: uniform
    const int ndict = static_cast<int>(nd);
    // offset -> code map: the ndict distinct table entries each claim a slot
    for (int i = threadIdx.x; i < kCodeLdsSlots; i += kBlock) key[i] = kCodeEmpty;
    __syncthreads();
    for (int i = threadIdx.x; i < ndict; i += kBlock) {
        const long long d = dict[i];
        const unsigned mask = kCodeLdsSlots - 1u;
        unsigned h = code_hash(d, 9);
        for (unsigned probe = 0; probe <= mask; ++probe, h = (h + 1u) & mask) {
            const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long *>(key + h),
                                                     static_cast<unsigned long long>(kCodeEmpty),
                                                     static_cast<unsigned long long>(d));
            if (static_cast<long long>(old) == kCodeEmpty) {
                code[h] = static_cast<unsigned char>(i);
                break;
            }
        }
    }
    __syncthreads();
    unsigned bad = 0;
    const int64_t T = (n_rows + kTileRows - 1) / kTileRows;
    CodeRows<P> nx;   // the next tile's row pointers, in flight while this one is worked on
    if (blockIdx.x < T) nx.load(n_rows, rp, static_cast<int64_t>(blockIdx.x) * kTileRows);
    for (int64_t tile = blockIdx.x; tile < T; tile += gridDim.x) {
        CodeTile<P, I> t;
        t.cols(nx, ci, row_of);
        if (tile + gridDim.x < T) nx.load(n_rows, rp, (tile + gridDim.x) * kTileRows);
        if (t.mapped) {
#pragma unroll
            for (int j = 0; j < kCodeBatch; ++j) {
                if (!t.valid(j)) continue;
                const int c = code_lookup(key, code, t.d[j]);
                if (c >= 0) codes[t.entry(j)] = static_cast<uint8_t>(c);
                else bad = 1;
            }
        } else {
            for (int64_t k = t.a; k < t.b; ++k) {
                const int c = code_lookup(key, code, static_cast<long long>(ci[k]) - t.row);
                if (c >= 0) codes[k] = static_cast<uint8_t>(c);
                else bad = 1;
            }
        }
        t.done();
    }
    if (bad) atomicOr(&words[1], 2u);
}

// Packed row pointers (with the codes only): tb[t] = the first entry of tile
// t (t <= T, tb[T] = nnz), ro[i] = row i's first entry less its tile's; an
// offset past 65535 sets words[2] and the plan keeps the plain row pointers.
template <typename P>
__global__ __launch_bounds__(kBlock) void k_rowpack(int64_t n_rows, const P *__restrict__ rp, int64_t *tb,
                                                    uint16_t *ro, unsigned *words) {
    if (words[1] != 0) return;   // no codes: uniform
    const int64_t T = (n_rows + kTileRows - 1) / kTileRows;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    unsigned bad = 0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n_rows; i += stride) {
        const int64_t r0 = (i / kTileRows) * kTileRows;
        const int64_t base = static_cast<int64_t>(rp[r0]);
        const int64_t off = static_cast<int64_t>(rp[i]) - base;
        if (off > 65535) bad = 1;
        ro[i] = static_cast<uint16_t>(off);
        if (i == r0) tb[i / kTileRows] = base;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) tb[T] = static_cast<int64_t>(rp[n_rows]);
    if (bad) atomicOr(&words[2], 1u);
}

// COO structure: row and column indices in range, rows non-decreasing.
template <typename I>
__global__ __launch_bounds__(kBlock) void k_coo_validate(int64_t n_rows, int64_t n_cols, int64_t nnz,
                                                         const I *__restrict__ row, const I *__restrict__ col,
                                                         unsigned *flags) {
    unsigned f = 0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; k < nnz; k += stride) {
        const int64_t r = static_cast<int64_t>(row[k]);
        const int64_t c = static_cast<int64_t>(col[k]);
        if (r < 0 || r >= n_rows) f |= VFLAG_BAD_FIRST;
        if (c < 0 || c >= n_cols) f |= VFLAG_BAD_COLUMN;
        if (k > 0 && r < static_cast<int64_t>(row[k - 1])) f |= VFLAG_UNSORTED;
    }
    if (f) atomicOr(flags, f);
}

// Row pointer of a row-sorted COO matrix: rp[i] = first entry whose row is
// >= i.  Entry k writes the pointers of the rows in (row[k-1], row[k]]; the
// first entry also those up to row[0], the last those after it.
template <typename I, typename P>
__global__ __launch_bounds__(kBlock) void k_coo_rowptr(int64_t n_rows, int64_t nnz, const I *__restrict__ row,
                                                       P *__restrict__ rp) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (nnz == 0) {
        for (int64_t i = gid; i <= n_rows; i += stride) rp[i] = 0;
        return;
    }
    for (int64_t k = gid; k < nnz; k += stride) {
        const int64_t r = static_cast<int64_t>(row[k]);
        const int64_t lo = k == 0 ? 0 : static_cast<int64_t>(row[k - 1]) + 1;
        for (int64_t i = lo; i <= r; ++i) rp[i] = static_cast<P>(k);
        if (k == nnz - 1)
            for (int64_t i = r + 1; i <= n_rows; ++i) rp[i] = static_cast<P>(nnz);
    }
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

// Random-gather probe: dst[i] = src[idx[i]] (indices and results streamed
// coalesced, the source read at random 8-byte positions).  Each thread keeps
// kGatherDepth gathers in flight (a row of an irregular SpMV keeps its row
// length), so the probe measures the memory system's rate, not one load's
// latency.
constexpr int kGatherDepth = 8;

__global__ __launch_bounds__(kBlock) void k_gather(const double *__restrict__ src, const int32_t *__restrict__ idx,
                                                   double *__restrict__ dst, int64_t m) {
    const int64_t span = static_cast<int64_t>(kBlock) * kGatherDepth;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * span;
    for (int64_t base = static_cast<int64_t>(blockIdx.x) * span + threadIdx.x; base < m; base += stride) {
        int32_t j[kGatherDepth];
        double v[kGatherDepth];
#pragma unroll
        for (int u = 0; u < kGatherDepth; ++u) {
            const int64_t e = base + static_cast<int64_t>(u) * kBlock;
            j[u] = e < m ? idx[e] : -1;
        }
#pragma unroll
        for (int u = 0; u < kGatherDepth; ++u) v[u] = j[u] >= 0 ? src[j[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < kGatherDepth; ++u) {
            const int64_t e = base + static_cast<int64_t>(u) * kBlock;
            if (e < m) dst[e] = v[u];
        }
    }
}

int grid_for(int64_t n, int per_thread, int cap) {
    const int64_t want = (n + static_cast<int64_t>(kBlock) * per_thread - 1) / (static_cast<int64_t>(kBlock) * per_thread);
    return static_cast<int>(want < 1 ? 1 : (want > cap ? cap : want));
}

}  // namespace

// ==================================================================== launchers
hipError_t launch_validate(const CsrDev &A, unsigned *flags, int max_grid, hipStream_t s) {
    const int64_t work = A.n_rows > A.nnz ? A.n_rows : A.nnz;
    const int grid = grid_for(work, 8, max_grid);
    return dispatch_idx(A, [&](auto rp, auto ci) {
        using P = pointee_t<decltype(rp)>;
        using I = pointee_t<decltype(ci)>;
        hipLaunchKernelGGL((k_validate<P, I>), dim3(grid), dim3(kBlock), 0, s, A.n_rows, A.n_cols, A.nnz, rp, ci, flags);
        return hipGetLastError();
    });
}

hipError_t launch_pattern_probe(const CsrDev &A, int step, long long *table, unsigned *words, int grid,
                                hipStream_t s) {
    if (step < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_code_clear, dim3(1), dim3(kBlock), 0, s, table, words);
    if (A.n_rows == 0) return hipGetLastError();
    return dispatch_idx(A, [&](auto rp, auto ci) {
        using P = pointee_t<decltype(rp)>;
        using I = pointee_t<decltype(ci)>;
        hipLaunchKernelGGL((k_code_collect<P, I>), dim3(grid), dim3(kBlock), 0, s, A.n_rows, rp, ci, step, table,
                           words);
        return hipGetLastError();
    });
}

hipError_t launch_code_build(const CsrDev &A, int step, long long *table, unsigned *words, void *codes_base,
                             int grid, hipStream_t s) {
    int64_t *dict = static_cast<int64_t *>(codes_base);
    uint8_t *codes = static_cast<uint8_t *>(codes_base) + kCodeDict * sizeof(int64_t);
    int64_t *tb = reinterpret_cast<int64_t *>(codes + code_bytes(A.nnz));
    if (step < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_code_clear, dim3(1), dim3(kBlock), 0, s, table, words);
    if (A.n_rows == 0) return hipGetLastError();
    return dispatch_idx(A, [&](auto rp, auto ci) {
        using P = pointee_t<decltype(rp)>;
        using I = pointee_t<decltype(ci)>;
        hipLaunchKernelGGL((k_code_collect<P, I>), dim3(grid), dim3(kBlock), 0, s, A.n_rows, rp, ci, step, table,
                           words);
        hipLaunchKernelGGL(k_code_table, dim3(1), dim3(kBlock), 0, s, table, words, dict);
        hipLaunchKernelGGL((k_code_encode<P, I>), dim3(grid), dim3(kBlock), 0, s, A.n_rows, rp, ci, dict, codes,
                           words);
        hipLaunchKernelGGL((k_rowpack<P>), dim3(grid), dim3(kBlock), 0, s, A.n_rows, rp, tb,
                           reinterpret_cast<uint16_t *>(tb + (A.n_rows + kTileRows - 1) / kTileRows + 1), words);
        return hipGetLastError();
    });
}

hipError_t launch_coo_validate(int64_t n_rows, int64_t n_cols, int64_t nnz, const void *row, const void *col,
                               int idx_t, unsigned *flags, int max_grid, hipStream_t s) {
    if (nnz == 0) return hipSuccess;
    const int grid = grid_for(nnz, 8, max_grid);
    if (idx_t == 0)
        hipLaunchKernelGGL(k_coo_validate<int32_t>, dim3(grid), dim3(kBlock), 0, s, n_rows, n_cols, nnz,
                           static_cast<const int32_t *>(row), static_cast<const int32_t *>(col), flags);
    else
        hipLaunchKernelGGL(k_coo_validate<int64_t>, dim3(grid), dim3(kBlock), 0, s, n_rows, n_cols, nnz,
                           static_cast<const int64_t *>(row), static_cast<const int64_t *>(col), flags);
    return hipGetLastError();
}

hipError_t launch_coo_rowptr(int64_t n_rows, int64_t nnz, const void *row, int idx_t, void *rp, int ptr_t,
                             hipStream_t s) {
    const int grid = grid_for(nnz > n_rows ? nnz : n_rows + 1, 8, kMaxGrid);
    if (idx_t == 0 && ptr_t == 0)
        hipLaunchKernelGGL((k_coo_rowptr<int32_t, int32_t>), dim3(grid), dim3(kBlock), 0, s, n_rows, nnz,
                           static_cast<const int32_t *>(row), static_cast<int32_t *>(rp));
    else if (idx_t == 0)
        hipLaunchKernelGGL((k_coo_rowptr<int32_t, int64_t>), dim3(grid), dim3(kBlock), 0, s, n_rows, nnz,
                           static_cast<const int32_t *>(row), static_cast<int64_t *>(rp));
    else if (ptr_t == 0)
        hipLaunchKernelGGL((k_coo_rowptr<int64_t, int32_t>), dim3(grid), dim3(kBlock), 0, s, n_rows, nnz,
                           static_cast<const int64_t *>(row), static_cast<int32_t *>(rp));
    else
        hipLaunchKernelGGL((k_coo_rowptr<int64_t, int64_t>), dim3(grid), dim3(kBlock), 0, s, n_rows, nnz,
                           static_cast<const int64_t *>(row), static_cast<int64_t *>(rp));
    return hipGetLastError();
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


hipError_t launch_cg_init(const CsrDev &A, const SpmvTune &t, const double *b, double *x, double *r, double *p,
                          SolveState *st, double *partials, double tau, int64_t max_iters, double *hist,
                          int64_t hist_cap, hipStream_t s) {
    EpiInit e{b, r, p, site(partials, SITE_INIT), 0.0, 0.0};
    hipError_t err = launch_family<double, double, double>(A, t, x, e, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_init_finish, dim3(1), dim3(kBlock), 0, s, st, site(partials, SITE_INIT), t.grid, tau,
                       max_iters, x, hist, hist_cap);
    return hipGetLastError();
}

hipError_t launch_fcg_init(const CsrDev &A, const SpmvTune &t, const double *b, double *x, const FcgBufs<double> &f,
                           SolveState *st, double *partials, double tau, int64_t max_iters, double *hist,
                           int64_t hist_cap, hipStream_t s) {
    fcg::EpiInit e{b, f.r[1], f.p[1], f.q[1], site(partials, SITE_INIT), 0.0, 0.0};
    hipError_t err = launch_family<double, double, double>(A, t, x, e, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_init_finish, dim3(1), dim3(kBlock), 0, s, st, site(partials, SITE_INIT), t.grid, tau,
                       max_iters, x, hist, hist_cap);
    return hipGetLastError();
}

hipError_t launch_fcg_step(const CsrDev &A, const SpmvTune &t, int j, const FcgBufs<double> &f, SolveState *st,
                           double *partials, hipStream_t s) {
    EpiFcg<double> e{};
    e.buf = f;
    e.st = st;
    e.part = site(partials, SITE_FCG);
    e.G = t.grid;
    e.j = j;
    return launch_family<double, double, double>(A, t, f.p[0], e, s);
}

hipError_t launch_fcg_step32(const CsrDev &A32, const SpmvTune &t, int j, const FcgBufs<float> &f, SolveState *st,
                             double *partials, hipStream_t s) {
    EpiFcg<float> e{};
    e.buf = f;
    e.st = st;
    e.part = site(partials, SITE_FCG);
    e.G = t.grid;
    e.j = j;
    if (A32.val_t == 1) return launch_family<float, float, float>(A32, t, f.p[0], e, s);
    if (A32.val_t == 3) return launch_family<bf16s, float, float>(A32, t, f.p[0], e, s);
    if (A32.val_t == 2) return launch_family<_Float16, float, float>(A32, t, f.p[0], e, s);
    return hipErrorInvalidValue;
}

hipError_t launch_fcg_ir_residual(const CsrDev &A, const SpmvTune &t, const double *b, const double *x,
                                  const FcgBufs<float> &f, float *d32, SolveState *in, double *partials,
                                  double tau_in, int64_t max_inner, double *out, hipStream_t s) {
    fcg::EpiIrResidual e{b, f.r[1], f.p[1], f.q[1], d32, site(partials, SITE_INIT), 0.0, 0.0, 0.0};
    hipError_t err = hipSuccess;
    if (A.val_t == 0) err = launch_family<double, double, double>(A, t, x, e, s);
    else if (A.val_t == 1) err = launch_family<float, double, double>(A, t, x, e, s);
    else return hipErrorInvalidValue;
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_ir_finish, dim3(1), dim3(kBlock), 0, s, in, site(partials, SITE_INIT), t.grid, tau_in,
                       max_inner, d32, out);
    return hipGetLastError();
}

hipError_t launch_cg_spmv_pq(const CsrDev &A, const SpmvTune &t, const double *p, double *q, SolveState *st,
                             double *partials, hipStream_t s) {
    EpiPq<double> e{q, p, st, site(partials, SITE_PQ), 0.0};
    return launch_family<double, double, double>(A, t, p, e, s);
}

hipError_t launch_cg_spmv_pq32(const CsrDev &A32, const SpmvTune &t, const float *p, float *q, SolveState *st,
                               double *partials, hipStream_t s) {
    EpiPq<float> e{q, p, st, site(partials, SITE_PQ), 0.0};
    if (A32.val_t == 1) return launch_family<float, float, float>(A32, t, p, e, s);
    if (A32.val_t == 3) return launch_family<bf16s, float, float>(A32, t, p, e, s);
    if (A32.val_t == 2) return launch_family<_Float16, float, float>(A32, t, p, e, s);
    return hipErrorInvalidValue;
}

hipError_t launch_cg_update(int64_t n, int grid, int spmv_grid, int j, double *r, const double *q, SolveState *st,
                            double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_update<double>, dim3(grid), dim3(kBlock), 0, s, n, r, q, st, site(partials, SITE_PQ),
                       spmv_grid, site(partials, SITE_RR), j);
    return hipGetLastError();
}

hipError_t launch_cg_update32(int64_t n, int grid, int spmv_grid, int j, float *r, const float *q, SolveState *st,
                              double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_update<float>, dim3(grid), dim3(kBlock), 0, s, n, r, q, st, site(partials, SITE_PQ),
                       spmv_grid, site(partials, SITE_RR), j);
    return hipGetLastError();
}

hipError_t launch_cg_pupdate(int64_t n, int grid, int j, const double *r, double *p, SolveState *st, double *partials,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_cg_pupdate<double>, dim3(grid), dim3(kBlock), 0, s, n, r, p, st, site(partials, SITE_RR),
                       grid, j);
    return hipGetLastError();
}

hipError_t launch_cg_pupdate32(int64_t n, int grid, int j, const float *r, float *p, SolveState *st,
                               double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_pupdate<float>, dim3(grid), dim3(kBlock), 0, s, n, r, p, st, site(partials, SITE_RR),
                       grid, j);
    return hipGetLastError();
}

hipError_t launch_ir_residual(const CsrDev &A, const SpmvTune &t, const double *b, const double *x, float *r32,
                              float *p32, float *d32, SolveState *in, double *partials, double tau_in,
                              int64_t max_inner, double *out, hipStream_t s) {
    EpiIrResidual e{b, r32, p32, d32, site(partials, SITE_INIT), 0.0, 0.0, 0.0};
    hipError_t err = hipSuccess;
    if (A.val_t == 0) err = launch_family<double, double, double>(A, t, x, e, s);
    else if (A.val_t == 1) err = launch_family<float, double, double>(A, t, x, e, s);
    else return hipErrorInvalidValue;
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_ir_finish, dim3(1), dim3(kBlock), 0, s, in, site(partials, SITE_INIT), t.grid, tau_in,
                       max_inner, d32, out);
    return hipGetLastError();
}

hipError_t launch_ir_correct(int64_t n, int grid, double *x, const float *d, hipStream_t s) {
    hipLaunchKernelGGL(k_ir_correct, dim3(grid), dim3(kBlock), 0, s, n, x, d);
    return hipGetLastError();
}

hipError_t launch_round_values(int64_t nnz, const double *src, void *dst, int to, int grid, hipStream_t s) {
    if (to == 3)   // BF16
        hipLaunchKernelGGL(k_round_values<bf16s>, dim3(grid), dim3(kBlock), 0, s, nnz, src, static_cast<bf16s *>(dst));
    else if (to == 2)   // F16
        hipLaunchKernelGGL(k_round_values<_Float16>, dim3(grid), dim3(kBlock), 0, s, nnz, src,
                           static_cast<_Float16 *>(dst));
    else if (to == 1)   // F32
        hipLaunchKernelGGL(k_round_values<float>, dim3(grid), dim3(kBlock), 0, s, nnz, src, static_cast<float *>(dst));
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_cg_chunk_end(SolveState *st, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_chunk_end, dim3(1), dim3(64), 0, s, st, count);
    return hipGetLastError();
}

hipError_t launch_cg_finalize(const CsrDev &A, const SpmvTune &t, const double *b, double *x_caller,
                              SolveState *st, double *partials, int true_residual, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_x, dim3(grid_for(A.n_rows, 8, kMaxGrid)), dim3(kBlock), 0, s, A.n_rows, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !true_residual) return e;
    EpiTrue et{b, st, site(partials, SITE_TRUE), 0.0};
    e = launch_family<double, double, double>(A, t, x_caller, et, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_true_finish, dim3(1), dim3(kBlock), 0, s, st, site(partials, SITE_TRUE), t.grid);
    return hipGetLastError();
}

hipError_t launch_gather(const double *src, const int32_t *idx, double *dst, int64_t m, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3(grid), dim3(kBlock), 0, s, src, idx, dst, m);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(kBlock), 0, s, static_cast<const uint4 *>(src),
                       static_cast<uint4 *>(dst), static_cast<int64_t>(bytes / 16));
    return hipGetLastError();
}

// The smaller residency of the plain and the p.q-fused SpMV of this type and
// tiling (plans time one of them; the other may run on the same launch shape).
int spmv_blocks_per_cu(const CsrDev &A, const SpmvTune &t) {
    int lo = 1 << 30;
    auto q = [&](auto kern) {
        int blocks = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, kBlock, 0) != hipSuccess) blocks = 1;
        lo = blocks < lo ? blocks : lo;
    };
    const bool i64 = A.idx_t != 0;
    const bool lr = A.max_row > kLongRow;   // plain-index kernels with the long-row pass
    auto q2 = [&](auto without, auto with) {
        if (lr) q(with);
        else q(without);
    };
    if (t.kind == 0 && t.codes && A.codes) {   // the coded instances the launch will use
        const bool pack = t.pack && A.rowpack;
        if (A.val_t == 0) {
            if (pack) {
                q(k_spmv_stream<double, RowPack, Code8, double, double, EpiPq<double>>);
                q(k_spmv_stream<double, RowPack, Code8, double, double, EpiPlain<double>>);
            } else {
                q(k_spmv_stream<double, int64_t, Code8, double, double, EpiPq<double>>);
                q(k_spmv_stream<double, int64_t, Code8, double, double, EpiPlain<double>>);
            }
        } else if (pack) {
            q(k_spmv_stream<float, RowPack, Code8, float, float, EpiPq<float>>);
            q(k_spmv_stream<float, RowPack, Code8, float, float, EpiPlain<float>>);
        } else {
            q(k_spmv_stream<float, int64_t, Code8, float, float, EpiPq<float>>);
            q(k_spmv_stream<float, int64_t, Code8, float, float, EpiPlain<float>>);
        }
    } else if (A.val_t == 0) {
        if (t.kind == 0) {
            if (i64) {
                q2(k_spmv_stream<double, int64_t, int64_t, double, double, EpiPq<double>>,
                   k_spmv_stream<double, int64_t, int64_t, double, double, EpiPq<double>, true>);
                q2(k_spmv_stream<double, int64_t, int64_t, double, double, EpiPlain<double>>,
                   k_spmv_stream<double, int64_t, int64_t, double, double, EpiPlain<double>, true>);
            } else {
                q2(k_spmv_stream<double, int64_t, int32_t, double, double, EpiPq<double>>,
                   k_spmv_stream<double, int64_t, int32_t, double, double, EpiPq<double>, true>);
                q2(k_spmv_stream<double, int64_t, int32_t, double, double, EpiPlain<double>>,
                   k_spmv_stream<double, int64_t, int32_t, double, double, EpiPlain<double>, true>);
            }
        } else {
            if (i64) {
                q(k_spmv_vector<double, int64_t, int64_t, double, double, EpiPq<double>>);
                q(k_spmv_vector<double, int64_t, int64_t, double, double, EpiPlain<double>>);
            } else {
                q(k_spmv_vector<double, int64_t, int32_t, double, double, EpiPq<double>>);
                q(k_spmv_vector<double, int64_t, int32_t, double, double, EpiPlain<double>>);
            }
        }
    } else {
        if (t.kind == 0) {
            q2(k_spmv_stream<float, int64_t, int32_t, float, float, EpiPlain<float>>,
               k_spmv_stream<float, int64_t, int32_t, float, float, EpiPlain<float>, true>);
            q2(k_spmv_stream<float, int64_t, int32_t, float, float, EpiPq<float>>,
               k_spmv_stream<float, int64_t, int32_t, float, float, EpiPq<float>, true>);
        } else {
            q(k_spmv_vector<float, int64_t, int32_t, float, float, EpiPlain<float>>);
            q(k_spmv_vector<float, int64_t, int32_t, float, float, EpiPq<float>>);
        }
    }
    return lo < 1 ? 1 : lo;
}

}  // namespace spk
