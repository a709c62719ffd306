// gfx950 kernels of the two further Krylov solves: CGS (the other solver of
// the paper's solver benchmarks, Section 6.2) and CG with the scalar Jacobi
// preconditioner (block size 1 in the configuration example of Section 3.5).
//
// Both reuse the SpMV tilings of spk_spmv.h with their own epilogues and keep
// the conventions of the CG kernels: one FP64 partial per workgroup, re-summed
// in a fixed order by every workgroup of the consuming launch (no atomics, no
// fences); per-iteration scalars in the state's 4-slot ring; every kernel
// returns at once once the stop flag is set.
//
// CGS, iteration k (Barrett et al. template, shadow residual rt = r_0):
//   dir(k)    : stop test on ||r_k|| (partials of the previous SpMV #2),
//               rho_k = rt.r_k, beta = rho_k / rho_{k-1};
//               u = r + beta q, p = u + beta (q + beta p)   (k = 0: u = p = r)
//   SpMV #1   : v = A p, partials of rt.v
//   update(k) : alpha = rho_k / rt.v; q = u - alpha v, uh = u + q, x += alpha uh
//   SpMV #2   : r -= alpha (A uh), partials of r.r and rt.r
// A chunk ends with check(c): the stop test of the chunk's last iteration,
// so the host reads a current verdict after every chunk.
//
// Jacobi PCG, iteration k (z = r / diag(A), kept implicit):
//   SpMV      : q = A p, partials of p.q   (the CG kernel)
//   update(k) : alpha = rho_k / p.q; r -= alpha q; partials of r.r and r.z
//   pupdate(k): x += alpha p; stop test on ||r||; rho_{k+1} = r.z;
//               p = z + beta p
#include "spk_launch.h"
#include "spk_spmv.h"

#include <cmath>

namespace spk {
namespace {

using namespace dev;
using namespace tile;

int grid_for(int64_t n, int per_thread, int cap) {
    const int64_t want = (n + static_cast<int64_t>(kBlock) * per_thread - 1) / (static_cast<int64_t>(kBlock) * per_thread);
    return static_cast<int>(want < 1 ? 1 : (want > cap ? cap : want));
}

// ------------------------------------------------------------------ CGS
// v = A p; partials of rt.v.
struct EpiCgsV {
    double *v;
    const double *rt;
    const SolveState *st;
    double *part;
    double acc;
    __device__ bool skip() const { return st->stop != STOP_RUNNING; }
    __device__ void row(int64_t i, double s) {
        v[i] = s;
        acc = fma(rt[i], s, acc);
    }
    __device__ void finish() {
        double w[1] = {acc};
        block_partial<1>(w, part);
    }
};

// r -= alpha (A uh); partials of r.r and rt.r.
struct EpiCgsR {
    double *r;
    const double *rt;
    const SolveState *st;
    double *part;
    double rr, rtr;
    __device__ bool skip() const { return st->stop != STOP_RUNNING; }
    __device__ void row(int64_t i, double s) {
        const double ri = fma(-st->alpha, s, r[i]);
        r[i] = ri;
        rr = fma(ri, ri, rr);
        rtr = fma(rt[i], ri, rtr);
    }
    __device__ void finish() {
        double w[2] = {rr, rtr};
        block_partial<2>(w, part);
    }
};

// Stop test of iteration k > 0 from the partials [r.r, rt.r] of the last
// SpMV #2; workgroup 0 records it.  Returns the verdict (same in every
// workgroup) and rho_k = rt.r_k.
__device__ __forceinline__ int cgs_test(SolveState *st, const double *part_rr, int G, int64_t k, double &rho) {
    double tot[2];
    sum_partials<2>(part_rr, G, tot);
    const double res = sqrt(tot[0]);
    rho = tot[1];
    int stop = STOP_RUNNING;
    if (!isfinite(res)) stop = STOP_NON_FINITE;
    else if (res <= st->thresh) stop = STOP_CONVERGED;
    else if (k >= st->max_iters) stop = STOP_MAX_ITERS;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->iter = k;
        st->resnorm = res;
        st->rho[k & 3] = rho;
        if (st->hist && k < st->hist_cap) st->hist[k] = res;
        if (stop != STOP_RUNNING) st->stop = stop;
    }
    return stop;
}

__global__ __launch_bounds__(kBlock) void k_cgs_dir(int64_t n, const double *__restrict__ r, double *__restrict__ u,
                                                    double *__restrict__ p, const double *__restrict__ q,
                                                    SolveState *st, const double *part_rr, int G_rr, int j) {
    if (st->stop != STOP_RUNNING) return;
    const int64_t k = st->base + j;
    double rho;
    if (k == 0) rho = st->rho[0];   // rt.r_0 = r_0.r_0, from the initial residual
    else if (cgs_test(st, part_rr, G_rr, k, rho) != STOP_RUNNING) return;
    if (!isfinite(rho) || rho == 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->stop = isfinite(rho) ? STOP_BREAKDOWN : STOP_NON_FINITE;
        return;
    }
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    using V2 = Vec16<double>::type;
    const int64_t nv = n / 2;
    const V2 *rv = reinterpret_cast<const V2 *>(r);
    V2 *uv = reinterpret_cast<V2 *>(u);
    V2 *pv = reinterpret_cast<V2 *>(p);
    const V2 *qv = reinterpret_cast<const V2 *>(q);
    if (k == 0) {
        for (int64_t i = gid; i < nv; i += stride) {
            const V2 ri = rv[i];
            uv[i] = ri;
            pv[i] = ri;
        }
        for (int64_t i = nv * 2 + gid; i < n; i += stride) {
            u[i] = r[i];
            p[i] = r[i];
        }
        return;
    }
    const double beta = rho / st->rho[(k - 1) & 3];
    for (int64_t i = gid; i < nv; i += stride) {
        const V2 ri = rv[i], qi = qv[i];
        V2 pi = pv[i], ui;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            ui[c] = fma(beta, qi[c], ri[c]);
            pi[c] = fma(beta, fma(beta, pi[c], qi[c]), ui[c]);
        }
        uv[i] = ui;
        pv[i] = pi;
    }
    for (int64_t i = nv * 2 + gid; i < n; i += stride) {
        const double ui = fma(beta, q[i], r[i]);
        u[i] = ui;
        p[i] = fma(beta, fma(beta, p[i], q[i]), ui);
    }
}

__global__ __launch_bounds__(kBlock) void k_cgs_update(int64_t n, const double *__restrict__ u,
                                                       const double *__restrict__ v, double *__restrict__ q,
                                                       double *__restrict__ uh, SolveState *st,
                                                       const double *part_v, int G_v, int j) {
    if (st->stop != STOP_RUNNING) return;
    const int64_t k = st->base + j;
    double tot[1];
    sum_partials<1>(part_v, G_v, tot);
    const double sigma = tot[0];
    if (!isfinite(sigma) || sigma == 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->pq = sigma;
            st->stop = isfinite(sigma) ? STOP_BREAKDOWN : STOP_NON_FINITE;
        }
        return;
    }
    const double alpha = st->rho[k & 3] / sigma;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->pq = sigma;
        st->alpha = alpha;
    }
    double *__restrict__ x = static_cast<double *>(st->x);
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    int64_t done = 0;
    if ((reinterpret_cast<uintptr_t>(x) & 15) == 0) {
        using V2 = Vec16<double>::type;
        const int64_t nv = n / 2;
        const V2 *uv = reinterpret_cast<const V2 *>(u);
        const V2 *vv = reinterpret_cast<const V2 *>(v);
        V2 *qv = reinterpret_cast<V2 *>(q);
        V2 *hv = reinterpret_cast<V2 *>(uh);
        V2 *xv = reinterpret_cast<V2 *>(x);
        for (int64_t i = gid; i < nv; i += stride) {
            const V2 ui = uv[i], vi = vv[i];
            V2 xi = xv[i], qi, hi;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                qi[c] = fma(-alpha, vi[c], ui[c]);
                hi[c] = ui[c] + qi[c];
                xi[c] = fma(alpha, hi[c], xi[c]);
            }
            qv[i] = qi;
            hv[i] = hi;
            xv[i] = xi;
        }
        done = nv * 2;
    }
    for (int64_t i = done + gid; i < n; i += stride) {
        const double qi = fma(-alpha, v[i], u[i]);
        const double hi = u[i] + qi;
        q[i] = qi;
        uh[i] = hi;
        x[i] = fma(alpha, hi, x[i]);
    }
}

// End of a chunk of `count` iterations: the stop test of the last one (the
// next chunk's first dir kernel repeats it, with the same outcome), then the
// chunk base advances.
__global__ __launch_bounds__(kBlock) void k_cgs_check(SolveState *st, const double *part_rr, int G_rr, int count) {
    if (st->stop == STOP_RUNNING) {
        double rho;
        (void)cgs_test(st, part_rr, G_rr, st->base + count, rho);
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) st->base += count;
}

// ------------------------------------------------------------------ Jacobi PCG
// dinv_i = 1 / (sum of row i's stored diagonal entries); flag[0] = 1 when
// some row has a zero or non-finite diagonal (no preconditioner then).
template <typename P, typename I>
__global__ __launch_bounds__(kBlock) void k_diag_inv(int64_t n, const P *__restrict__ rp, const I *__restrict__ ci,
                                                     const double *__restrict__ va, double *__restrict__ dinv,
                                                     unsigned *flag) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    bool bad = false;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
        double d = 0.0;
        for (int64_t k = static_cast<int64_t>(rp[i]); k < static_cast<int64_t>(rp[i + 1]); ++k)
            if (static_cast<int64_t>(ci[k]) == i) d += va[k];
        bad |= (d == 0.0 || !isfinite(d));
        dinv[i] = 1.0 / d;
    }
    if (bad) flag[0] = 1u;   // plain store: every writer stores the same value
}

// Right preconditioning by M = diag(A): the scaled copy of the values,
// out_k = val_k / d_{col_k} (as val_k * dinv_{col_k}).
template <typename I>
__global__ __launch_bounds__(kBlock) void k_scale_cols(int64_t nnz, const I *__restrict__ ci,
                                                       const double *__restrict__ va, const double *__restrict__ dinv,
                                                       double *__restrict__ out) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; k < nnz; k += stride)
        out[k] = va[k] * dinv[static_cast<int64_t>(ci[k])];
}

// to_u = 1: x <- D x (= x / dinv), the unknown of the right-preconditioned
// system; to_u = 0: x <- D^{-1} u (= u * dinv).
__global__ __launch_bounds__(kBlock) void k_jacobi_vec(int64_t n, double *__restrict__ x,
                                                       const double *__restrict__ dinv, int to_u) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride)
        x[i] = to_u ? x[i] / dinv[i] : x[i] * dinv[i];
}

// r = b - A x, p = z = dinv r; partials of r.r, r.z and b.b.
struct EpiPcgInit {
    const double *b, *dinv;
    double *r, *p;
    double *part;
    double rr, rz, bb;
    __device__ bool skip() const { return false; }
    __device__ void row(int64_t i, double s) {
        const double bi = b[i];
        const double ri = bi - s;
        const double zi = ri * dinv[i];
        r[i] = ri;
        p[i] = zi;
        rr = fma(ri, ri, rr);
        rz = fma(ri, zi, rz);
        bb = fma(bi, bi, bb);
    }
    __device__ void finish() {
        double w[3] = {rr, rz, bb};
        block_partial<3>(w, part);
    }
};

// Initial verdict.  Order as in the definition: non-finite ||b||, then an
// unusable diagonal (breakdown, x untouched), then b = 0, then the tests on
// r_0.
__global__ __launch_bounds__(kBlock) void k_pcg_init_finish(SolveState *st, const double *part, int G, double tau,
                                                            int64_t max_iters, double *x, double *hist,
                                                            int64_t hist_cap, const unsigned *bad_diag) {
    double tot[3];
    sum_partials<3>(part, G, tot);
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
    const double bn = sqrt(tot[2]);
    st->bnorm = bn;
    st->thresh = tau * bn;
    if (!isfinite(bn)) {
        st->stop = STOP_NON_FINITE;
        st->resnorm = bn;
    } else if (bad_diag[0] != 0) {
        st->stop = STOP_BREAKDOWN;
        st->resnorm = __builtin_nan("");
    } else if (bn == 0.0) {
        st->zero_x = 1;
        st->stop = STOP_CONVERGED;
        st->resnorm = 0.0;
        st->true_resnorm = 0.0;
        st->rho[0] = 0.0;
        if (hist && hist_cap > 0) hist[0] = 0.0;
    } else {
        const double res = sqrt(tot[0]);
        const double rho = tot[1];
        st->rho[0] = rho;
        st->resnorm = res;
        if (hist && hist_cap > 0) hist[0] = res;
        if (!isfinite(rho) || !isfinite(res)) st->stop = STOP_NON_FINITE;
        else if (res <= tau * bn) st->stop = STOP_CONVERGED;
        else if (max_iters <= 0) st->stop = STOP_MAX_ITERS;
    }
}

// alpha = rho_k / p.q; r -= alpha q; partials of r.r and r.z (z = dinv r).
__global__ __launch_bounds__(kBlock) void k_pcg_update(int64_t n, double *__restrict__ r, const double *__restrict__ q,
                                                       const double *__restrict__ dinv, SolveState *st,
                                                       const double *part_pq, int G_pq, double *part_rr, int j) {
    if (st->stop != STOP_RUNNING) return;
    const int64_t k = st->base + j;
    double tot[1];
    sum_partials<1>(part_pq, G_pq, tot);
    const double pq = tot[0];
    if (!isfinite(pq) || pq <= 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->pq = pq;
            st->stop = isfinite(pq) ? STOP_BREAKDOWN : STOP_NON_FINITE;
        }
        return;
    }
    const double alpha = st->rho[k & 3] / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->pq = pq;
        st->alpha = alpha;
    }
    double rr = 0.0, rz = 0.0;
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    using V2 = Vec16<double>::type;
    const int64_t nv = n / 2;
    V2 *rv = reinterpret_cast<V2 *>(r);
    const V2 *qv = reinterpret_cast<const V2 *>(q);
    const V2 *dv = reinterpret_cast<const V2 *>(dinv);
    for (int64_t i = gid; i < nv; i += stride) {
        V2 ri = rv[i];
        const V2 qi = qv[i], di = dv[i];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            ri[c] = fma(-alpha, qi[c], ri[c]);
            rr = fma(ri[c], ri[c], rr);
            rz = fma(ri[c], ri[c] * di[c], rz);
        }
        rv[i] = ri;
    }
    for (int64_t i = nv * 2 + gid; i < n; i += stride) {
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        rr = fma(ri, ri, rr);
        rz = fma(ri, ri * dinv[i], rz);
    }
    double w[2] = {rr, rz};
    block_partial<2>(w, part_rr);
}

// x += alpha p; stop test on ||r_{k+1}||; rho_{k+1} = r.z; beta; p = z + beta p.
__global__ __launch_bounds__(kBlock) void k_pcg_pupdate(int64_t n, const double *__restrict__ r,
                                                        const double *__restrict__ dinv, double *__restrict__ p,
                                                        SolveState *st, const double *part_rr, int G_rr, int j) {
    if (st->stop != STOP_RUNNING) return;
    const int64_t k = st->base + j;
    double tot[2];
    sum_partials<2>(part_rr, G_rr, tot);
    const double res = sqrt(tot[0]);
    const double rho_new = tot[1];
    const int64_t k1 = k + 1;
    int stop = STOP_RUNNING;
    if (!isfinite(rho_new) || !isfinite(res)) stop = STOP_NON_FINITE;
    else if (res <= st->thresh) stop = STOP_CONVERGED;
    else if (k1 >= st->max_iters) stop = STOP_MAX_ITERS;
    const double beta = rho_new / st->rho[k & 3];
    const double alpha = st->alpha;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->iter = k1;
        st->resnorm = res;
        st->rho[k1 & 3] = rho_new;
        if (st->hist && k1 < st->hist_cap) st->hist[k1] = res;
        if (stop != STOP_RUNNING) st->stop = stop;
    }
    const bool more = stop == STOP_RUNNING;
    double *__restrict__ x = static_cast<double *>(st->x);
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    int64_t done = 0;
    if ((reinterpret_cast<uintptr_t>(x) & 15) == 0) {
        using V2 = Vec16<double>::type;
        const int64_t nv = n / 2;
        V2 *xv = reinterpret_cast<V2 *>(x);
        V2 *pv = reinterpret_cast<V2 *>(p);
        const V2 *rv = reinterpret_cast<const V2 *>(r);
        const V2 *dv = reinterpret_cast<const V2 *>(dinv);
        for (int64_t i = gid; i < nv; i += stride) {
            V2 xi = xv[i], pi = pv[i];
#pragma unroll
            for (int c = 0; c < 2; ++c) xi[c] = fma(alpha, pi[c], xi[c]);
            xv[i] = xi;
            if (more) {
                const V2 ri = rv[i], di = dv[i];
#pragma unroll
                for (int c = 0; c < 2; ++c) pi[c] = fma(beta, pi[c], ri[c] * di[c]);
                pv[i] = pi;
            }
        }
        done = nv * 2;
    }
    for (int64_t i = done + gid; i < n; i += stride) {
        const double pi = p[i];
        x[i] = fma(alpha, pi, x[i]);
        if (more) p[i] = fma(beta, pi, r[i] * dinv[i]);
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_cgs_dir(int64_t n, int grid, int spmv_grid, int j, const double *r, double *u, double *p,
                          const double *q, SolveState *st, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_cgs_dir, dim3(grid), dim3(kBlock), 0, s, n, r, u, p, q, st, site(partials, SITE_RR),
                       spmv_grid, j);
    return hipGetLastError();
}

hipError_t launch_cgs_spmv_v(const CsrDev &A, const SpmvTune &t, const double *p, double *v, const double *rt,
                             SolveState *st, double *partials, hipStream_t s) {
    EpiCgsV e{v, rt, st, site(partials, SITE_PQ), 0.0};
    return launch_family<double, double, double>(A, t, p, e, s);
}

hipError_t launch_cgs_update(int64_t n, int grid, int spmv_grid, int j, const double *u, const double *v, double *q,
                             double *uh, SolveState *st, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_cgs_update, dim3(grid), dim3(kBlock), 0, s, n, u, v, q, uh, st, site(partials, SITE_PQ),
                       spmv_grid, j);
    return hipGetLastError();
}

hipError_t launch_cgs_spmv_r(const CsrDev &A, const SpmvTune &t, const double *uh, double *r, const double *rt,
                             SolveState *st, double *partials, hipStream_t s) {
    EpiCgsR e{r, rt, st, site(partials, SITE_RR), 0.0, 0.0};
    return launch_family<double, double, double>(A, t, uh, e, s);
}

hipError_t launch_cgs_check(SolveState *st, double *partials, int spmv_grid, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_cgs_check, dim3(1), dim3(kBlock), 0, s, st, site(partials, SITE_RR), spmv_grid, count);
    return hipGetLastError();
}

hipError_t launch_diag_inv(const CsrDev &A, double *dinv, unsigned *flag, hipStream_t s) {
    if (A.n_rows == 0) return hipSuccess;
    const int grid = grid_for(A.n_rows, 4, kMaxGrid);
    return dispatch_idx(A, [&](auto rp, auto ci) {
        using P = pointee_t<decltype(rp)>;
        using I = pointee_t<decltype(ci)>;
        hipLaunchKernelGGL((k_diag_inv<P, I>), dim3(grid), dim3(kBlock), 0, s, A.n_rows, rp, ci,
                           static_cast<const double *>(A.va), dinv, flag);
        return hipGetLastError();
    });
}

hipError_t launch_scale_cols(const CsrDev &A, const double *dinv, double *out, hipStream_t s) {
    if (A.nnz == 0) return hipSuccess;
    const int grid = grid_for(A.nnz, 8, kMaxGrid);
    if (A.idx_t == 0)
        hipLaunchKernelGGL(k_scale_cols<int32_t>, dim3(grid), dim3(kBlock), 0, s, A.nnz,
                           static_cast<const int32_t *>(A.ci), static_cast<const double *>(A.va), dinv, out);
    else
        hipLaunchKernelGGL(k_scale_cols<int64_t>, dim3(grid), dim3(kBlock), 0, s, A.nnz,
                           static_cast<const int64_t *>(A.ci), static_cast<const double *>(A.va), dinv, out);
    return hipGetLastError();
}

hipError_t launch_jacobi_vec(int64_t n, double *x, const double *dinv, int to_u, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_jacobi_vec, dim3(grid_for(n, 8, kMaxGrid)), dim3(kBlock), 0, s, n, x, dinv, to_u);
    return hipGetLastError();
}

hipError_t launch_pcg_init(const CsrDev &A, const SpmvTune &t, const double *b, double *x, const double *dinv,
                           const unsigned *bad_diag, double *r, double *p, SolveState *st, double *partials,
                           double tau, int64_t max_iters, double *hist, int64_t hist_cap, hipStream_t s) {
    EpiPcgInit e{b, dinv, r, p, site(partials, SITE_INIT), 0.0, 0.0, 0.0};
    hipError_t err = launch_family<double, double, double>(A, t, x, e, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_pcg_init_finish, dim3(1), dim3(kBlock), 0, s, st, site(partials, SITE_INIT), t.grid, tau,
                       max_iters, x, hist, hist_cap, bad_diag);
    return hipGetLastError();
}

hipError_t launch_pcg_update(int64_t n, int grid, int spmv_grid, int j, double *r, const double *q,
                             const double *dinv, SolveState *st, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_update, dim3(grid), dim3(kBlock), 0, s, n, r, q, dinv, st, site(partials, SITE_PQ),
                       spmv_grid, site(partials, SITE_RR), j);
    return hipGetLastError();
}

hipError_t launch_pcg_pupdate(int64_t n, int grid, int j, const double *r, const double *dinv, double *p,
                              SolveState *st, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_pupdate, dim3(grid), dim3(kBlock), 0, s, n, r, dinv, p, st, site(partials, SITE_RR),
                       grid, j);
    return hipGetLastError();
}

}  // namespace spk
