// The fused CG step: CG with one SpMV-based pass per iteration, shared by the
// per-launch step (spk_kernels.hip) and the persistent solve
// (spk_persist.hip).
//
// Step k (k = 0, 1, ...) of the loop:
//   decision (k >= 1), identical in every workgroup: the partial sums step
//     k-1 left give p.q, r.q, q.q and r.r of iteration k-1; stop when
//     ||r_{k-1}|| <= tau ||b|| (k - 1 >= 1; r_0 is tested by the initial
//     residual), at the iteration cap, when p.q <= 0 (breakdown) or on a
//     non-finite value; otherwise alpha = rho / p.q with rho = r_{k-1}.r_{k-1},
//     rho_k from rho - 2 alpha r.q + alpha^2 q.q (the squared norm of
//     r_{k-1} - alpha q_{k-1}, expanded) and beta = rho_k / rho;
//   rows: r_k = r_{k-1} - alpha q_{k-1}, p_k = r_k + beta p_{k-1},
//     x_k = x_{k-1} + alpha p_{k-1}, q_k = A p_k, with p_k formed at every
//     gathered column from the previous step's r, q and p by the same
//     expression as for the row itself (so the gathered and the stored p_k
//     agree bit for bit); r_k, p_k and q_k go to the other buffer of each
//     pair; partials of p_k.q_k, r_k.q_k, q_k.q_k and r_k.r_k.
// Step 0 runs with alpha = beta = 0 on r_0 and zeroed p and q, so it forms
// p_0 = r_0 and q_0 = A p_0.  The stop test is the textbook one on the
// recomputed r_k.r_k, taken one step later (step k+1 returns at once when r_k
// meets it); only beta uses the expanded form, because r_k is complete
// nowhere until the step ends.  Per iteration the loop reads A once, gathers
// r, q and p, reads and writes x and writes r, p and q: 8 n vector words
// against 10 n for a three-launch iteration.
#pragma once

#include "spk_device.h"

namespace spk {
namespace fcg {

using namespace dev;

template <typename T>
struct Gather {
    const T *__restrict__ r;
    const T *__restrict__ q;
    const T *__restrict__ p;
    T alpha, beta;
    __device__ __forceinline__ T operator()(int64_t c) const { return fma(beta, p[c], fma(-alpha, q[c], r[c])); }
};

// The stop reason at the start of step done + 1 from iteration done's sums
// tot = {p.q, r.q, q.q, r.r}; when going on (STOP_RUNNING), alpha and beta.
__device__ __forceinline__ int decide(const double (&tot)[4], int64_t done, double thresh, int64_t max_iters,
                                      double &alpha, double &beta) {
    const double pq = tot[0], rq = tot[1], qq = tot[2], rho = tot[3];
    if (!isfinite(rho)) return STOP_NON_FINITE;
    if (done >= 1 && sqrt(rho) <= thresh) return STOP_CONVERGED;
    if (done >= max_iters) return STOP_MAX_ITERS;
    if (!isfinite(pq)) return STOP_NON_FINITE;
    if (pq <= 0.0) return STOP_BREAKDOWN;
    alpha = rho / pq;
    const double rho_k = rho - 2.0 * alpha * rq + alpha * alpha * qq;
    beta = rho_k > 0.0 ? rho_k / rho : 0.0;
    return STOP_RUNNING;
}

// What the state records of iteration done (one thread).
__device__ __forceinline__ void record(SolveState *st, const double (&tot)[4], int64_t done) {
    const double res = sqrt(tot[3]);
    st->iter = done;
    st->resnorm = res;
    st->rho[done & 3] = tot[3];
    st->pq = tot[0];
    if (done >= 1 && st->hist && done < st->hist_cap) st->hist[done] = res;
}

// The row work of one step: the epilogue of its SpMV.
template <typename T>
struct Rows {
    const T *ro, *qo, *po;   // iteration k-1 (gathered)
    T *rn, *pn, *qn;         // iteration k
    T *x;
    T alpha, beta;
    double acc[4];
    // step k reads buffer (k + 1) & 1 of each pair and writes buffer k & 1
    // (selected by value: an index into the pairs would keep them in memory)
    __device__ __forceinline__ void bind(const FcgBufs<T> &f, T *x_, int64_t k) {
        const bool odd = (k & 1) != 0;
        ro = odd ? f.r[0] : f.r[1];
        qo = odd ? f.q[0] : f.q[1];
        po = odd ? f.p[0] : f.p[1];
        rn = odd ? f.r[1] : f.r[0];
        pn = odd ? f.p[1] : f.p[0];
        qn = odd ? f.q[1] : f.q[0];
        x = x_;
        alpha = beta = T(0);
        acc[0] = acc[1] = acc[2] = acc[3] = 0.0;
    }
    __device__ Gather<T> gather() const { return Gather<T>{ro, qo, po, alpha, beta}; }
    // the row's own entries of the previous vectors and of x, loaded with
    // the tile (the tile loop issues pre() beside its DMA)
    struct Own {
        T p, q, r, x;
    };
    __device__ __forceinline__ Own pre(int64_t i) const { return Own{po[i], qo[i], ro[i], x[i]}; }
    template <class C>
    __device__ __forceinline__ void row(int64_t i, C s) { row(i, s, pre(i)); }
    template <class C>
    __device__ __forceinline__ void row(int64_t i, C s, const Own &o) {
        const T qk = static_cast<T>(s);
        const T pold = o.p;
        const T rk = fma(-alpha, o.q, o.r);
        const T pk = fma(beta, pold, rk);
        x[i] = fma(alpha, pold, o.x);
        rn[i] = rk;
        pn[i] = pk;
        qn[i] = qk;
        const double qd = static_cast<double>(qk), rd = static_cast<double>(rk);
        acc[0] = fma(static_cast<double>(pk), qd, acc[0]);
        acc[1] = fma(rd, qd, acc[1]);
        acc[2] = fma(qd, qd, acc[2]);
        acc[3] = fma(rd, rd, acc[3]);
    }
};

// Initial residual of the loop: r_0 = b - A x (into r), p = q = 0; partials
// of r.r and b.b.
struct EpiInit {
    const double *b;
    double *r, *p, *q;
    double *part;
    double rr, bb;
    __device__ bool skip() const { return false; }
    __device__ void row(int64_t i, double s) {
        const double bi = b[i];
        const double ri = bi - s;
        r[i] = ri;
        p[i] = 0.0;
        q[i] = 0.0;
        rr = fma(ri, ri, rr);
        bb = fma(bi, bi, bb);
    }
    __device__ void finish() {
        double v[2] = {rr, bb};
        block_partial<2>(v, part);
    }
};

// Refinement step before an FP32 inner loop: r = b - A x in FP64, the inner
// right-hand side r32 = fl32(r), the inner p, q and d zeroed; partials of
// ||r||^2 (FP64), ||r32||^2 (FP64 sums of the rounded values) and ||b||^2.
struct EpiIrResidual {
    const double *b;
    float *r32, *p32, *q32, *d32;
    double *part;
    double rr, rr32, bb;
    __device__ bool skip() const { return false; }
    __device__ void row(int64_t i, double s) {
        const double bi = b[i];
        const double ri = bi - s;
        const float ri32 = static_cast<float>(ri);
        r32[i] = ri32;
        p32[i] = 0.0f;
        q32[i] = 0.0f;
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

}  // namespace fcg
}  // namespace spk
