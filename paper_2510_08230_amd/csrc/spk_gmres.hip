// gfx950 kernels of restarted GMRES(m), the solver of the paper's usage
// examples (Listings 1-2, Krylov dimension 30) and of its solver benchmarks
// (Section 6.2).
//
// Arnoldi orthogonalisation is classical Gram-Schmidt applied twice, with
// the second projection delayed by one pass: each pass is one streaming
// kernel over the basis (multi-dot and multi-axpy, HBM-bound), and a step
// reads the basis twice instead of three times.  At step j the basis holds
// the finished vectors q_0..q_{j-1} (Q_j) and, in slot j, the candidate
// u_j = Q_j a + nu q_j: once orthogonalised, with a (its components along
// Q_j) and nu known but the second projection not yet subtracted.
//   SpMV   : w = A u_j
//   passA  : partials of b_t = q_t . w (t < j) and of u_j . w
//   reduce : b
//   coef   : with Qb = [Q_j, q_j] and A Q_j = Qb Hu (earlier columns),
//            A q_j = (w - Qb e) / nu, e = Hu a; its projections
//            h = Qb^T A q_j = (Qb^T w - e) / nu, where q_j . w =
//            (u_j . w - a . b) / nu; u_{j+1} = w / nu - Qb d, d = e / nu + h
//   passB  : q_j = (u_j - Q_j a) / nu written over u_j; u_{j+1} into slot
//            j+1; partials of a' = Qb^T u_{j+1} and of ||u_{j+1}||^2
//   reduce : a'
//   final  : nu' = sqrt(||u_{j+1}||^2 - ||a'||^2); column j of Hu is h + a'
//            with nu' below it (A q_j = Qb (h + a') + nu' q_{j+1}); earlier
//            rotations, a new rotation, g, the residual estimate |g_{j+1}|,
//            the stop test
// A cycle starts with the residual r = b - A x written into slot 0 as the
// candidate u_0 (a empty, nu = ||r||) and ends with the triangular solve
// R y = g and x += Q y over the columns built.  Kernels return at once when
// the solve has stopped or the cycle is done, so the host can enqueue a
// whole cycle and poll once.
//
// The basis, w and x are of type T: double for the FP64 solve, float for the
// inner solve of mixed-precision refinement (FP32/BF16/FP16 matrix values).
// Every dot product, norm and Gram-Schmidt combination is formed in FP64 from
// the stored values and rounded once to T; Hu, H, g and the rotations are FP64.
#include "spk_launch.h"
#include "spk_spmv.h"

#include <cmath>

namespace spk {
namespace {

using namespace dev;
using namespace tile;

__device__ __forceinline__ bool gm_idle(const SolveState *st, const GmresState *gs) {
    return st->stop != STOP_RUNNING || gs->cycle_done != 0;
}

// r = b - A x into v_0; partials of r.r and b.b.
template <typename T>
struct EpiGmRes {
    const T *b;
    T *v0;
    const SolveState *st;
    double *part;
    double rr, bb;
    __device__ bool skip() const { return st->stop != STOP_RUNNING; }
    template <class C>
    __device__ void row(int64_t i, C s) {
        const double bi = static_cast<double>(b[i]);
        const T ri = static_cast<T>(bi - static_cast<double>(s));
        v0[i] = ri;
        rr = fma(static_cast<double>(ri), static_cast<double>(ri), rr);
        bb = fma(bi, bi, bb);
    }
    __device__ void finish() {
        double w[2] = {rr, bb};
        block_partial<2>(w, part);
    }
};

// w = A u_j.
template <typename T>
struct EpiGmW {
    T *w;
    const SolveState *st;
    const GmresState *gs;
    __device__ bool skip() const { return gm_idle(st, gs); }
    template <class C>
    __device__ void row(int64_t i, C s) { w[i] = static_cast<T>(s); }
    __device__ void finish() {}
};

// r = b into v_0 when x = 0 (the first cycle of a refinement's inner solve,
// which starts from d = 0): the partials EpiGmRes would give, without the SpMV.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gm_residual_zero(int64_t n, const T *__restrict__ b, T *__restrict__ v0,
                                                             const SolveState *st, double *part) {
    if (st->stop != STOP_RUNNING) return;
    double rr = 0.0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
        const T bi = b[i];
        v0[i] = bi;
        rr = fma(static_cast<double>(bi), static_cast<double>(bi), rr);
    }
    double w[2] = {rr, rr};
    block_partial<2>(w, part);
}

// Solve set-up (one thread): the state fields every later kernel reads.
__global__ void k_gm_begin(SolveState *st, GmresState *gs, void *x, double *hist, int64_t hist_cap,
                           int64_t max_iters) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
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
    gs->cycle_done = 0;
    gs->used = 0;
}

// Cycle start: ||b||, beta = ||r||, the stop tests on r, g = beta e_0.
__global__ __launch_bounds__(kBlock) void k_gm_cycle_start(SolveState *st, GmresState *gs, const double *part, int G,
                                                           double tau, int m) {
    if (st->stop != STOP_RUNNING) {
        if (threadIdx.x == 0) gs->cycle_done = 1;
        return;
    }
    double tot[2];
    sum_partials<2>(part, G, tot);
    if (threadIdx.x != 0) return;
    const double bn = sqrt(tot[1]);
    const double beta = sqrt(tot[0]);
    st->bnorm = bn;
    st->thresh = tau * bn;
    int stop = STOP_RUNNING;
    if (!isfinite(bn)) {
        stop = STOP_NON_FINITE;
        st->resnorm = bn;
    } else if (bn == 0.0) {
        st->zero_x = 1;
        stop = STOP_CONVERGED;
        st->resnorm = 0.0;
        st->true_resnorm = 0.0;
        if (st->iter == 0 && st->hist && st->hist_cap > 0) st->hist[0] = 0.0;
    } else {
        st->resnorm = beta;
        if (st->iter == 0 && st->hist && st->hist_cap > 0) st->hist[0] = beta;
        if (!isfinite(beta)) stop = STOP_NON_FINITE;
        else if (beta <= tau * bn) stop = STOP_CONVERGED;
        else if (st->iter >= st->max_iters) stop = STOP_MAX_ITERS;
    }
    gs->used = 0;
    gs->cycle_done = stop != STOP_RUNNING;
    gs->nu = beta;   // candidate u_0 = r = beta q_0
    gs->g[0] = beta;
    for (int i = 1; i <= m; ++i) gs->g[i] = 0.0;
    if (stop != STOP_RUNNING) st->stop = stop;
}

// The vector passes move packs of K consecutive elements per lane and load
// (per-element 4-byte loads left the FP32 passes bound by load issue at
// about 2.2 TB/s).  Two shapes, chosen by the basis bucket NV:
//  * streaming (passA and passB up to NV = 8): 16-byte packs, each vector's
//    pack combined as it arrives; low register use, high occupancy.
//  * load-all-first (larger NV, and update_x): a thread issues the loads of
//    every basis vector it needs before combining them, so one pack of all J
//    vectors is in flight at once.  K trades that register footprint against
//    occupancy: pack_len<T, NV, B>() is the widest pack (16 bytes at most)
//    with NV * K * B <= 256, B = sizeof(T) up to NV = 16, else 8 (the
//    compiler holds FP32 values converted to FP64).
// passB keeps every finished vector's pack until u_{j+1} is formed (its dot
// products need it); it splits the basis over several lanes per pack to keep
// that footprint small (see k_gm_passB), and passA takes the same split for
// all but the FP64 small-basis bucket (k_gm_passA_split).
// Basis columns sit ld = gm_ld(n) elements apart (16-byte aligned); the last
// pack of a vector is loaded element by element when n is not a multiple
// of K.
template <typename T, int NV, int B>
constexpr int pack_len() {
    int k = 16 / static_cast<int>(sizeof(T));
    while (k > 1 && NV * k * B > 256) k /= 2;
    return k;
}

template <typename T, int K>
__device__ __forceinline__ void ld_pack(const T *__restrict__ p, int64_t i0, int64_t n, T (&o)[K]) {
    if constexpr (K == 1) {
        o[0] = p[i0];
    } else {
        typedef T vk __attribute__((ext_vector_type(K)));
        if (i0 + K <= n) {
            const vk v = *reinterpret_cast<const vk *>(p + i0);
#pragma unroll
            for (int e = 0; e < K; ++e) o[e] = v[e];
        } else {
#pragma unroll
            for (int e = 0; e < K; ++e) o[e] = i0 + e < n ? p[i0 + e] : T(0);
        }
    }
}

template <typename T, int K>
__device__ __forceinline__ void st_pack(T *__restrict__ p, int64_t i0, int64_t n, const T (&o)[K]) {
    if constexpr (K == 1) {
        p[i0] = o[0];
    } else {
        typedef T vk __attribute__((ext_vector_type(K)));
        if (i0 + K <= n) {
            vk v;
#pragma unroll
            for (int e = 0; e < K; ++e) v[e] = o[e];
            *reinterpret_cast<vk *>(p + i0) = v;
        } else {
#pragma unroll
            for (int e = 0; e < K; ++e)
                if (i0 + e < n) p[i0 + e] = o[e];
        }
    }
}

// Basis vector t of the Krylov block.
template <typename T>
__device__ __forceinline__ const T *vec(const T *V, int64_t ld, int t) { return V + static_cast<int64_t>(t) * ld; }

// First pass of step j: partials of b_t = q_t . w (t < j) and of u_j . w
// (t = j; the candidate sits in slot j).
template <typename T, int NV>
__global__ __launch_bounds__(kBlock) void k_gm_passA(int64_t n, int64_t ld, const T *__restrict__ V,
                                                     const T *__restrict__ w, int j, const SolveState *st,
                                                     const GmresState *gs, double *part) {
    if (gm_idle(st, gs)) return;
    constexpr bool stream = NV <= 8;
    constexpr int K = stream ? 16 / static_cast<int>(sizeof(T)) : pack_len<T, NV, (NV >= 32 ? 8 : sizeof(T))>();
    double acc[NV];
#pragma unroll
    for (int t = 0; t < NV; ++t) acc[t] = 0.0;
    const int64_t np = (n + K - 1) / K;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; q < np; q += stride) {
        const int64_t i0 = q * K;
        T wv[K];
        ld_pack<T, K>(w, i0, n, wv);
        if constexpr (stream) {
#pragma unroll
            for (int t = 0; t < NV; ++t) {
                if (t <= j) {
                    T vt[K];
                    ld_pack<T, K>(vec(V, ld, t), i0, n, vt);
#pragma unroll
                    for (int e = 0; e < K; ++e)
                        acc[t] = fma(static_cast<double>(wv[e]), static_cast<double>(vt[e]), acc[t]);
                }
            }
        } else {
            T vt[NV][K];
#pragma unroll
            for (int t = 0; t < NV; ++t) {
                if (t <= j) {
                    ld_pack<T, K>(vec(V, ld, t), i0, n, vt[t]);
                } else {
#pragma unroll
                    for (int e = 0; e < K; ++e) vt[t][e] = T(0);
                }
            }
#pragma unroll
            for (int t = 0; t < NV; ++t) {
                if (t <= j) {
#pragma unroll
                    for (int e = 0; e < K; ++e)
                        acc[t] = fma(static_cast<double>(wv[e]), static_cast<double>(vt[t][e]), acc[t]);
                }
            }
        }
    }
    block_partial<NV>(acc, part);
}

// Partial sums of one coefficient per workgroup: out[t] = sum of part row t.
__global__ __launch_bounds__(kBlock) void k_gm_reduce(const double *part, int G, double *out, const SolveState *st,
                                                      const GmresState *gs) {
    if (gm_idle(st, gs)) return;
    const int t = blockIdx.x;
    double tot[1];
    sum_partials<1>(part + static_cast<int64_t>(t) * kMaxGrid, G, tot);
    if (threadIdx.x == 0) out[t] = tot[0];
}

// Step coefficients (one thread; J <= 33 terms): h (column j before the
// delayed correction) and d (u_{j+1} = w / nu - sum d_t q_t, t <= j).
__global__ void k_gm_coef(const SolveState *st, GmresState *gs, int j) {
    if (gm_idle(st, gs) || threadIdx.x != 0 || blockIdx.x != 0) return;
    const double inv = 1.0 / gs->nu;
    double qwj = gs->b[j];   // u_j . w  ->  q_j . w
    for (int t = 0; t < j; ++t) qwj = fma(-gs->a[t], gs->b[t], qwj);
    qwj *= inv;
    for (int s = 0; s <= j; ++s) {
        // e_s = sum_{t < j} Hu[s][t] a_t (Hu[s][t] = 0 for s > t + 1)
        double e = 0.0;
        for (int t = s > 0 ? s - 1 : 0; t < j; ++t) e = fma(gs->Hu[s * kMaxKrylov + t], gs->a[t], e);
        const double qw = s < j ? gs->b[s] : qwj;
        const double h = (qw - e) * inv;
        gs->h[s] = h;
        gs->d[s] = fma(e, inv, h);
    }
}

// Second pass of step j: q_j = (u_j - Q_j a) / nu over the candidate,
// u_{j+1} = w / nu - Q_j d - d_j q_j into slot j + 1, partials of
// a'_t = q_t . u_{j+1} (t <= j, rows 0..NV-1) and of ||u_{j+1}||^2 (row NV).
// uj (slot j, read and written) and un (slot j + 1) do not overlap the
// finished vectors read through V.
//
// The dot products need every finished vector's pack until u_{j+1} is known,
// so one lane holding all J of them ran at one or two waves per SIMD.  Here S
// lanes share a pack: lane group g of a wave (64 / S lanes) holds the vectors
// t = u S + g only; the groups' partial combinations sum_t a_t q_t and
// sum_t d_t q_t are added across the S lanes of a pack (the same sum in
// every lane: the exchange adds in one fixed pattern), group 0 stores the
// pack's q_j and u_{j+1}, and every lane accumulates the dot products of its
// own vectors.
// Lanes per pack in passB by value type and basis bucket, measured on
// stencil7_ns N=215 (mean us per working launch, one lane / two / four):
// FP64 NV = 8: 116 / 107 / 115, NV = 16: - / 246 / 235, NV = 32: - / - /
// 404; FP32 (the GMRES-IR basis) NV = 8: - / 55 / 80, NV = 16: - / 133 /
// 120.  (Combining each vector's pack as it arrived, which kept one load in
// flight per lane, took 106, 241 and 436 for FP64 and 61 and 132 for FP32
// at the best split.)
template <typename T, int NV>
constexpr int passb_split() {
    return NV <= 8 ? 2 : 4;
}

template <typename T, int NV, int S>
constexpr int passb_pack() {
    int k = 16 / static_cast<int>(sizeof(T));
    while (k > 1 && (NV / S) * k * static_cast<int>(sizeof(T)) > 128) k /= 2;
    return k;
}

// passA with the basis split over S lanes per pack, as passB: lane group g
// of a wave holds the vectors t = u S + g (t <= j), each lane sums its
// vectors' products with w over its pack, and the workgroup partial of
// vector t is its group's sum followed by the four waves in order.
template <typename T, int NV, int S>
__global__ __launch_bounds__(kBlock) void k_gm_passA_split(int64_t n, int64_t ld, const T *__restrict__ V,
                                                           const T *__restrict__ w, int j, const SolveState *st,
                                                           const GmresState *gs, double *part) {
    if (gm_idle(st, gs)) return;
    static_assert(NV % S == 0 && (S == 1 || S == 2 || S == 4), "lane split");
    constexpr int NS = NV / S;
    constexpr int LP = 64 / S;
    constexpr int K = passb_pack<T, NV, S>();
    __shared__ double sh[NV][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int g = lane / LP, pl = lane % LP;
    double acc[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) acc[u] = 0.0;
    const int64_t np = (n + K - 1) / K;
    const int64_t per_block = static_cast<int64_t>(kBlock / 64) * LP;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * per_block;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * per_block + wid * LP + pl; q < np; q += stride) {
        const int64_t i0 = q * K;
        T wv[K], vt[NS][K];
        ld_pack<T, K>(w, i0, n, wv);
#pragma unroll
        for (int u = 0; u < NS; ++u)
            if (u * S + g <= j) ld_pack<T, K>(vec(V, ld, u * S + g), i0, n, vt[u]);
#pragma unroll
        for (int u = 0; u < NS; ++u)
            if (u * S + g <= j) {
#pragma unroll
                for (int e = 0; e < K; ++e)
                    acc[u] = fma(static_cast<double>(wv[e]), static_cast<double>(vt[u][e]), acc[u]);
            }
    }
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        double v = acc[u];
#pragma unroll
        for (int off = LP / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (pl == 0) sh[u * S + g][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int t = threadIdx.x;
        double v = sh[t][0];
#pragma unroll
        for (int w2 = 1; w2 < kBlock / 64; ++w2) v += sh[t][w2];
        part[static_cast<size_t>(t) * kMaxGrid + blockIdx.x] = v;
    }
}

template <typename T, int NV, int S>
__global__ __launch_bounds__(kBlock) void k_gm_passB(int64_t n, int64_t ld, const T *__restrict__ V,
                                                     T *__restrict__ uj, T *__restrict__ un,
                                                     const T *__restrict__ w, int j, const SolveState *st,
                                                     const GmresState *gs, double *part) {
    if (gm_idle(st, gs)) return;
    static_assert(NV % S == 0 && (S == 1 || S == 2 || S == 4), "lane split");
    constexpr int NS = NV / S;    // vectors per lane
    constexpr int LP = 64 / S;    // packs per wave and round
    constexpr int K = passb_pack<T, NV, S>();
    __shared__ double ca[NV], cd[NV + 1];
    __shared__ double sh[NV + 1][kBlock / 64];
    if (threadIdx.x < NV) ca[threadIdx.x] = static_cast<int>(threadIdx.x) < j ? gs->a[threadIdx.x] : 0.0;
    if (threadIdx.x <= NV) cd[threadIdx.x] = static_cast<int>(threadIdx.x) <= j ? gs->d[threadIdx.x] : 0.0;
    __syncthreads();
    const double inv = 1.0 / gs->nu;
    const double dj = cd[j];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int g = lane / LP, pl = lane % LP;
    double acc[NS], accn = 0.0;
#pragma unroll
    for (int u = 0; u < NS; ++u) acc[u] = 0.0;
    const int64_t np = (n + K - 1) / K;
    const int64_t per_block = static_cast<int64_t>(kBlock / 64) * LP;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * per_block;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * per_block + wid * LP + pl; q < np; q += stride) {
        const int64_t i0 = q * K;
        // every load of the round is issued before the first use, so the
        // lane's packs are in flight together
        T vt[NS][K], wv[K], uv[K];
        ld_pack<T, K>(w, i0, n, wv);
        ld_pack<T, K>(uj, i0, n, uv);
#pragma unroll
        for (int u = 0; u < NS; ++u)
            if (u * S + g < j) ld_pack<T, K>(vec(V, ld, u * S + g), i0, n, vt[u]);
        double pq[K], pn[K];
#pragma unroll
        for (int e = 0; e < K; ++e) pq[e] = pn[e] = 0.0;
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const int t = u * S + g;
            if (t < j) {
#pragma unroll
                for (int e = 0; e < K; ++e) {
                    const double v = static_cast<double>(vt[u][e]);
                    pq[e] = fma(ca[t], v, pq[e]);
                    pn[e] = fma(cd[t], v, pn[e]);
                }
            }
        }
        if constexpr (S > 1) {
#pragma unroll
            for (int off = LP; off < 64; off <<= 1) {
#pragma unroll
                for (int e = 0; e < K; ++e) {
                    pq[e] += __shfl_xor(pq[e], off, 64);
                    pn[e] += __shfl_xor(pn[e], off, 64);
                }
            }
        }
        T qv[K], nv[K];
#pragma unroll
        for (int e = 0; e < K; ++e) {
            const double qd = static_cast<double>(uv[e]) - pq[e];
            const double nd = fma(static_cast<double>(wv[e]), inv, -pn[e]);
            qv[e] = static_cast<T>(qd * inv);
            nv[e] = static_cast<T>(fma(-dj, static_cast<double>(qv[e]), nd));
        }
        if (g == 0) {
            st_pack<T, K>(uj, i0, n, qv);
            st_pack<T, K>(un, i0, n, nv);
        }
#pragma unroll
        for (int e = 0; e < K; ++e) {
            const double u1 = static_cast<double>(nv[e]);
#pragma unroll
            for (int u = 0; u < NS; ++u) {
                const int t = u * S + g;
                if (t < j) acc[u] = fma(static_cast<double>(vt[u][e]), u1, acc[u]);
                else if (t == j) acc[u] = fma(static_cast<double>(qv[e]), u1, acc[u]);
            }
            if (g == 0) accn = fma(u1, u1, accn);
        }
    }
    // workgroup partials: per vector t = u S + g the sum over its lane group,
    // then the four waves in order; row NV: ||u_{j+1}||^2 from group 0
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        double v = acc[u];
#pragma unroll
        for (int off = LP / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (pl == 0) sh[u * S + g][wid] = v;
    }
    {
        double v = accn;
#pragma unroll
        for (int off = LP / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) sh[NV][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x <= NV) {
        const int t = threadIdx.x;
        double v = sh[t][0];
#pragma unroll
        for (int w2 = 1; w2 < kBlock / 64; ++w2) v += sh[t][w2];
        part[static_cast<size_t>(t) * kMaxGrid + blockIdx.x] = v;
    }
}

// End of step j (one workgroup; thread 0 does the scalar work): nu' from
// ||u_{j+1}||^2 (partials row nvrow) and a'; column j of Hu and of the
// rotated H; earlier rotations, a new rotation, g, the residual estimate and
// the stop test.
__global__ __launch_bounds__(kBlock) void k_gm_final(SolveState *st, GmresState *gs, const double *part, int G,
                                                     int nvrow, int j, int m) {
    if (gm_idle(st, gs)) return;
    double tot[1];
    sum_partials<1>(part + static_cast<int64_t>(nvrow) * kMaxGrid, G, tot);
    if (threadIdx.x != 0) return;
    double s2 = 0.0;
    for (int t = 0; t <= j; ++t) s2 = fma(gs->a[t], gs->a[t], s2);
    const double hn = sqrt(fmax(tot[0] - s2, 0.0));
    double *H = gs->H;
    for (int t = 0; t <= j; ++t) {
        const double c = gs->h[t] + gs->a[t];
        gs->Hu[t * kMaxKrylov + j] = c;
        H[t * kMaxKrylov + j] = c;
    }
    gs->Hu[(j + 1) * kMaxKrylov + j] = hn;
    for (int t = 0; t < j; ++t) {
        const double a = H[t * kMaxKrylov + j], c = H[(t + 1) * kMaxKrylov + j];
        H[t * kMaxKrylov + j] = gs->cs[t] * a + gs->sn[t] * c;
        H[(t + 1) * kMaxKrylov + j] = -gs->sn[t] * a + gs->cs[t] * c;
    }
    const double a = H[j * kMaxKrylov + j];
    const double d = hypot(a, hn);
    double c = 1.0, s = 0.0;
    if (d != 0.0) {
        c = a / d;
        s = hn / d;
    }
    gs->cs[j] = c;
    gs->sn[j] = s;
    H[j * kMaxKrylov + j] = c * a + s * hn;
    H[(j + 1) * kMaxKrylov + j] = 0.0;
    gs->g[j + 1] = -s * gs->g[j];
    gs->g[j] = c * gs->g[j];
    const int64_t k = st->iter + 1;
    const double res = fabs(gs->g[j + 1]);
    st->iter = k;
    st->resnorm = res;
    if (st->hist && k < st->hist_cap) st->hist[k] = res;
    int stop = STOP_RUNNING;
    if (!isfinite(res)) stop = STOP_NON_FINITE;
    else if (res <= st->thresh) stop = STOP_CONVERGED;
    else if (k >= st->max_iters) stop = STOP_MAX_ITERS;
    gs->used = j + 1;
    gs->nu = hn;   // the candidate u_{j+1} = Qb a' + nu' q_{j+1}
    if (stop != STOP_RUNNING || hn == 0.0 || j + 1 == m) gs->cycle_done = 1;
    if (stop != STOP_RUNNING) st->stop = stop;
}

// R y = g by back substitution over the columns built (one thread).
__global__ void k_gm_solve(const SolveState *st, GmresState *gs) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int used = gs->used;
    if (st->stop == STOP_NON_FINITE || used == 0) return;
    for (int i = used - 1; i >= 0; --i) {
        double s = gs->g[i];
        for (int t = i + 1; t < used; ++t) s -= gs->H[i * kMaxKrylov + t] * gs->y[t];
        gs->y[i] = s / gs->H[i * kMaxKrylov + i];
    }
}

// x += V y over the columns built, added column by column (in FP64, then
// rounded once to T).  x is the caller's vector: packed only when aligned
// to the pack.
template <typename T, int NV>
__global__ __launch_bounds__(kBlock) void k_gm_update_x(int64_t n, int64_t ld, const T *__restrict__ V,
                                                        const SolveState *st, const GmresState *gs) {
    const int used = gs->used;
    if (st->stop == STOP_NON_FINITE || used == 0) return;
    constexpr int K = pack_len<T, NV, 8>();
    __shared__ double y[NV];
    if (threadIdx.x < NV) y[threadIdx.x] = static_cast<int>(threadIdx.x) < used ? gs->y[threadIdx.x] : 0.0;
    __syncthreads();
    T *__restrict__ x = static_cast<T *>(st->x);
    const bool aligned = (reinterpret_cast<uintptr_t>(x) % (K * sizeof(T))) == 0;
    const int64_t np = (n + K - 1) / K;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; q < np; q += stride) {
        const int64_t i0 = q * K;
        T xv[K], vt[NV][K];
        if (aligned) {
            ld_pack<T, K>(x, i0, n, xv);
        } else {
#pragma unroll
            for (int e = 0; e < K; ++e) xv[e] = i0 + e < n ? x[i0 + e] : T(0);
        }
#pragma unroll
        for (int t = 0; t < NV; ++t) {
            if (t < used) {
                ld_pack<T, K>(vec(V, ld, t), i0, n, vt[t]);
            } else {
#pragma unroll
                for (int e = 0; e < K; ++e) vt[t][e] = T(0);
            }
        }
        double xd[K];
#pragma unroll
        for (int e = 0; e < K; ++e) xd[e] = static_cast<double>(xv[e]);
#pragma unroll
        for (int t = 0; t < NV; ++t)
#pragma unroll
            for (int e = 0; e < K; ++e) xd[e] = fma(y[t], static_cast<double>(vt[t][e]), xd[e]);
#pragma unroll
        for (int e = 0; e < K; ++e) xv[e] = static_cast<T>(xd[e]);
        if (aligned) {
            st_pack<T, K>(x, i0, n, xv);
        } else {
#pragma unroll
            for (int e = 0; e < K; ++e)
                if (i0 + e < n) x[i0 + e] = xv[e];
        }
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers
static int nv_bucket(int J) { return J <= 8 ? 8 : (J <= 16 ? 16 : 32); }

// SpMV with a GMRES epilogue: FP64 vectors need F64 values; FP32 vectors
// take F32, BF16 or F16 values.
template <typename T, class Epi>
static hipError_t gm_spmv(const CsrDev &A, const SpmvTune &t, const T *x, const Epi &e, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        if (A.val_t != 0) return hipErrorInvalidValue;
        return launch_family<double, double, double>(A, t, x, e, s);
    } else {
        if (A.val_t == 1) return launch_family<float, float, float>(A, t, x, e, s);
        if (A.val_t == 3) return launch_family<bf16s, float, float>(A, t, x, e, s);
        if (A.val_t == 2) return launch_family<_Float16, float, float>(A, t, x, e, s);
        return hipErrorInvalidValue;
    }
}

hipError_t launch_gm_begin(SolveState *st, GmresState *gs, void *x, double *hist, int64_t hist_cap,
                           int64_t max_iters, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_begin, dim3(1), dim3(64), 0, s, st, gs, x, hist, hist_cap, max_iters);
    return hipGetLastError();
}

template <typename T>
static hipError_t cycle_start_t(const CsrDev &A, const SpmvTune &t, const void *b, const void *x, void *V,
                                SolveState *st, GmresState *gs, double *partials, double tau, int m, hipStream_t s) {
    EpiGmRes<T> e{static_cast<const T *>(b), static_cast<T *>(V), st, site(partials, SITE_INIT), 0.0, 0.0};
    hipError_t err = gm_spmv<T>(A, t, static_cast<const T *>(x), e, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_gm_cycle_start, dim3(1), dim3(kBlock), 0, s, st, gs, site(partials, SITE_INIT), t.grid, tau,
                       m);
    return hipGetLastError();
}

hipError_t launch_gm_cycle_start(const CsrDev &A, const SpmvTune &t, const void *b, const void *x, void *V,
                                 SolveState *st, GmresState *gs, double *partials, double tau, int m, bool fp32,
                                 hipStream_t s) {
    return fp32 ? cycle_start_t<float>(A, t, b, x, V, st, gs, partials, tau, m, s)
                : cycle_start_t<double>(A, t, b, x, V, st, gs, partials, tau, m, s);
}

hipError_t launch_gm_cycle_start_zero(int64_t n, int grid, const void *b, void *V, SolveState *st, GmresState *gs,
                                      double *partials, double tau, int m, bool fp32, hipStream_t s) {
    if (fp32)
        hipLaunchKernelGGL(k_gm_residual_zero<float>, dim3(grid), dim3(kBlock), 0, s, n, static_cast<const float *>(b),
                           static_cast<float *>(V), st, site(partials, SITE_INIT));
    else
        hipLaunchKernelGGL(k_gm_residual_zero<double>, dim3(grid), dim3(kBlock), 0, s, n,
                           static_cast<const double *>(b), static_cast<double *>(V), st, site(partials, SITE_INIT));
    hipLaunchKernelGGL(k_gm_cycle_start, dim3(1), dim3(kBlock), 0, s, st, gs, site(partials, SITE_INIT), grid, tau, m);
    return hipGetLastError();
}

template <typename T>
static hipError_t step_spmv_t(const CsrDev &A, const SpmvTune &t, const void *V, void *w, int j,
                              const SolveState *st, const GmresState *gs, hipStream_t s) {
    EpiGmW<T> e{static_cast<T *>(w), st, gs};
    return gm_spmv<T>(A, t, static_cast<const T *>(V) + static_cast<int64_t>(j) * gm_ld(A.n_rows), e, s);
}

hipError_t launch_gm_step_spmv(const CsrDev &A, const SpmvTune &t, const void *V, void *w, int j,
                               const SolveState *st, const GmresState *gs, bool fp32, hipStream_t s) {
    return fp32 ? step_spmv_t<float>(A, t, V, w, j, st, gs, s) : step_spmv_t<double>(A, t, V, w, j, st, gs, s);
}

// passA form by value type and basis bucket: 0 = one lane per pack
// (k_gm_passA), S > 0 = S lanes per pack (k_gm_passA_split).  Measured on
// stencil7_ns N=215 (mean us per working launch; one lane per pack, then
// the split form with one / two / four lanes): FP64 NV = 8: 81 / 89 / 85 /
// 82, NV = 16: 199 / 198 / 195 / 186, NV = 32: 331 / 330 / 321 / 322; FP32
// NV = 8: 38 / 37 / 35 / 35, NV = 16: 153 / 100 / 96 / 90, NV = 32: 143 /
// 142 / 136 / 128.
template <typename T, int NV>
constexpr int passa_split() { return sizeof(T) == 8 && NV <= 8 ? 0 : 4; }

template <typename T, int NV>
static void launch_passA(int grid, int64_t n, int64_t ld, const T *V, const T *w, int j, const SolveState *st,
                         const GmresState *gs, double *gpart, hipStream_t s) {
    if constexpr (passa_split<T, NV>() == 0)
        hipLaunchKernelGGL((k_gm_passA<T, NV>), dim3(grid), dim3(kBlock), 0, s, n, ld, V, w, j, st, gs, gpart);
    else
        hipLaunchKernelGGL((k_gm_passA_split<T, NV, passa_split<T, NV>()>), dim3(grid), dim3(kBlock), 0, s, n, ld, V,
                           w, j, st, gs, gpart);
}

template <typename T>
static hipError_t step_rest_t(int64_t n, int grid, T *V, T *w, int j, int m, SolveState *st, GmresState *gs,
                              double *gpart, hipStream_t s) {
    const int J = j + 1;
    const int nv = nv_bucket(J);
    const int64_t ld = gm_ld(n);
    T *uj = V + static_cast<int64_t>(j) * ld;
    T *un = V + static_cast<int64_t>(j + 1) * ld;
    if (nv == 8) launch_passA<T, 8>(grid, n, ld, V, w, j, st, gs, gpart, s);
    else if (nv == 16) launch_passA<T, 16>(grid, n, ld, V, w, j, st, gs, gpart, s);
    else launch_passA<T, 32>(grid, n, ld, V, w, j, st, gs, gpart, s);
    hipLaunchKernelGGL(k_gm_reduce, dim3(J), dim3(kBlock), 0, s, gpart, grid, &gs->b[0], st, gs);
    hipLaunchKernelGGL(k_gm_coef, dim3(1), dim3(64), 0, s, st, gs, j);
    // passB: lanes per pack by basis bucket
    if (nv == 8)
        hipLaunchKernelGGL((k_gm_passB<T, 8, passb_split<T, 8>()>), dim3(grid), dim3(kBlock), 0, s, n, ld, V, uj, un,
                           w, j, st, gs, gpart);
    else if (nv == 16)
        hipLaunchKernelGGL((k_gm_passB<T, 16, passb_split<T, 16>()>), dim3(grid), dim3(kBlock), 0, s, n, ld, V, uj,
                           un, w, j, st, gs, gpart);
    else
        hipLaunchKernelGGL((k_gm_passB<T, 32, passb_split<T, 32>()>), dim3(grid), dim3(kBlock), 0, s, n, ld, V, uj,
                           un, w, j, st, gs, gpart);
    hipLaunchKernelGGL(k_gm_reduce, dim3(J), dim3(kBlock), 0, s, gpart, grid, &gs->a[0], st, gs);
    hipLaunchKernelGGL(k_gm_final, dim3(1), dim3(kBlock), 0, s, st, gs, gpart, grid, nv, j, m);
    return hipGetLastError();
}

hipError_t launch_gm_step_rest(int64_t n, int grid, void *V, void *w, int j, int m, SolveState *st, GmresState *gs,
                               double *gpart, bool fp32, hipStream_t s) {
    return fp32 ? step_rest_t<float>(n, grid, static_cast<float *>(V), static_cast<float *>(w), j, m, st, gs, gpart, s)
                : step_rest_t<double>(n, grid, static_cast<double *>(V), static_cast<double *>(w), j, m, st, gs,
                                      gpart, s);
}

template <typename T>
static hipError_t cycle_end_t(int64_t n, int grid, int m, const T *V, SolveState *st, GmresState *gs, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_solve, dim3(1), dim3(64), 0, s, st, gs);
    const int nv = nv_bucket(m);
    const int64_t ld = gm_ld(n);
    if (nv == 8) hipLaunchKernelGGL((k_gm_update_x<T, 8>), dim3(grid), dim3(kBlock), 0, s, n, ld, V, st, gs);
    else if (nv == 16) hipLaunchKernelGGL((k_gm_update_x<T, 16>), dim3(grid), dim3(kBlock), 0, s, n, ld, V, st, gs);
    else hipLaunchKernelGGL((k_gm_update_x<T, 32>), dim3(grid), dim3(kBlock), 0, s, n, ld, V, st, gs);
    return hipGetLastError();
}

hipError_t launch_gm_cycle_end(int64_t n, int grid, int m, const void *V, SolveState *st, GmresState *gs, bool fp32,
                               hipStream_t s) {
    return fp32 ? cycle_end_t<float>(n, grid, m, static_cast<const float *>(V), st, gs, s)
                : cycle_end_t<double>(n, grid, m, static_cast<const double *>(V), st, gs, s);
}

}  // namespace spk
