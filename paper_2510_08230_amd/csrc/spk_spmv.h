// The SpMV tilings and their launch helper, shared by the kernel sources.
//
//   * LDS-staged row tiles: a workgroup owns 256 consecutive rows; it streams
//     the tile's values and column indices from HBM into LDS with fully
//     coalesced loads (one contiguous nnz range per tile), then each thread
//     reduces one row from LDS while gathering x.  Tiles whose nnz exceed the
//     LDS capacity fall back to direct loads.
//   * lanes-per-row vector kernel: 2^k lanes of a wave64 share a row.
// Both hand each row sum to an epilogue object (row(i, s), finish()), which is
// where the solvers fuse their elementwise work and dot-product partials.
// The LDS tiles also read a plan's compressed index arrays: one-byte column
// codes (I = Code8: column = row + offset table[code], the table in LDS) and
// packed row pointers (P = RowPack: an int64 per tile, a uint16 per row);
// row sums keep their order, so the products equal the plain ones bit for bit.
#pragma once

#include "spk_device.h"

#include <algorithm>
#include <type_traits>
#include <utility>

namespace spk {
namespace tile {

using namespace dev;

// Partial-sum slab k of the workspace.
inline double *site(double *partials, int k) { return partials + static_cast<size_t>(k) * kSiteWidth * kMaxGrid; }

template <typename T>
struct Vec16 {
    static constexpr int W = 16 / sizeof(T);
    typedef T type __attribute__((ext_vector_type(W)));
};

// Entry range [a, b) of one row (long-row pass: the bounds are loaded again
// rather than kept live through the per-lane row loop).
template <typename P>
__device__ __forceinline__ void row_range(const P *__restrict__ rp, int64_t n, int64_t row, int64_t &a, int64_t &b) {
    a = static_cast<int64_t>(rp[row]);
    b = static_cast<int64_t>(rp[row + 1]);
}

template <>
__device__ __forceinline__ void row_range<RowPack>(const RowPack *__restrict__ rp, int64_t n, int64_t row, int64_t &a,
                                                   int64_t &b) {
    const int64_t *tb = reinterpret_cast<const int64_t *>(rp);
    const uint16_t *ro = reinterpret_cast<const uint16_t *>(tb + (n + kTileRows - 1) / kTileRows + 1);
    const int64_t tile = row / kTileRows;
    const int64_t r1 = min((tile + 1) * static_cast<int64_t>(kTileRows), n);
    a = tb[tile] + ro[row];
    b = row + 1 < r1 ? tb[tile] + ro[row + 1] : tb[tile + 1];
}

// The rows of the tile at r0 whose flag lng is set (rows longer than the
// long-row limit), summed one at a time by the whole workgroup in ascending
// row order -- each thread a strided share in storage order, then the wave
// sums and the four wave totals in a fixed order -- and handed to epi.row by
// the row's own thread.  Every thread of the workgroup calls this (it
// synchronises); the flags go through LDS as one ballot per wave, so nothing
// of the per-lane row loop stays live for it.  val(k) / cix(k): entry k's
// value and stored column (read from global memory, also for a tile staged
// in LDS: one call site keeps the kernel's register count down).
template <typename C, typename P, class Gx, class D, class Epi, class Val, class Cix>
__device__ __forceinline__ void long_rows(bool lng, const P *__restrict__ rp, int64_t n, int64_t r0, const Gx &gx,
                                          const D &col, Epi &epi, const Val &val, const Cix &cix) {
    __shared__ unsigned long long s_mask[kBlock / 64];
    __shared__ C s_red[kBlock / 64];
    const unsigned long long m = __ballot(lng);
    if ((threadIdx.x & 63) == 0) s_mask[threadIdx.x >> 6] = m;
    __syncthreads();
#pragma unroll 1
    for (int w = 0; w < kBlock / 64; ++w) {
        unsigned long long left = s_mask[w];
        while (left != 0) {   // the same in every thread
            const int i = w * 64 + __builtin_ctzll(left);
            left &= left - 1;
            const int64_t row = r0 + i;
            int64_t ra, rb;
            row_range(rp, n, row, ra, rb);
            C acc = 0;
#pragma unroll 1
            for (int64_t k = ra + threadIdx.x; k < rb; k += kBlock)
                acc = fma(static_cast<C>(widen(val(k))), static_cast<C>(gx(col(cix(k), row))), acc);
            acc = wave_sum(acc);
            if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
            __syncthreads();
            if (static_cast<int>(threadIdx.x) == i) {
                C t = s_red[0];
#pragma unroll
                for (int v = 1; v < kBlock / 64; ++v) t += s_red[v];
                epi.row(row, t);
            }
            __syncthreads();   // s_red is reused by the next long row
        }
    }
    __syncthreads();           // s_mask is rewritten by the next tile
}

// Epilogue operands loaded with the tile: an epilogue that reads a vector at
// its row (p_i for p.q, b_i for a residual) may provide pre(i), returning
// that value, and row(i, sum, value).  The tile loop then issues the load
// beside the tile's DMA, whose wait covers it, instead of after the row sum,
// where it would add a memory round trip to every tile.
template <class Epi, class = void>
struct HasPre : std::false_type {};
template <class Epi>
struct HasPre<Epi, std::void_t<decltype(std::declval<const Epi &>().pre(int64_t(0)))>> : std::true_type {};

struct NoPre {};

template <class Epi>
__device__ __forceinline__ auto pre_of(const Epi &epi, int64_t i) {
    if constexpr (HasPre<Epi>::value) return epi.pre(i);
    else return NoPre{};
}

template <class Epi, class C, class Pv>
__device__ __forceinline__ void emit_row(Epi &epi, int64_t i, C sum, const Pv &pv) {
    if constexpr (std::is_same_v<Pv, NoPre>) epi.row(i, sum);
    else epi.row(i, sum, pv);
}

// LDS-staged row tiles: DMA the tile's values and columns into LDS, then one
// thread per row reduces from LDS while gathering x.  Occupancy (several
// workgroups per CU) overlaps one workgroup's DMA with another's gathers.
// The tile loop of the LDS-staged SpMV, shared by the per-launch kernel and the
// persistent CG kernel: calls epi.row(row, sum) for every row of the tiles
// this workgroup visits.  lv / lc: the workgroup's LDS staging buffers.
// LR (the matrix has rows longer than kLongRow entries): those rows are
// summed by the whole workgroup (long_rows), so a hub row does not serialise
// its tile on one lane.  A compile-time switch: the pass costs registers, and
// with it in every instance the kernels without hub rows lost a workgroup per
// CU.
template <typename V, typename P, typename I, typename C, bool LR, class Gx, class Epi, class D = ColPlain>
__device__ __forceinline__ void spmv_tiles_lds(int64_t n, int64_t nnz, const P *__restrict__ rp,
                                               const I *__restrict__ ci, const V *__restrict__ va, const Gx &gx,
                                               int remap, int nt, int pf, Epi &epi, u32x4 *lv, u32x4 *lc,
                                               const D &col = D{}, uint32_t walkers = 0) {
    const V *sv = reinterpret_cast<const V *>(lv);
    const I *sc = reinterpret_cast<const I *>(lc);
    const int64_t T = (n + kTileRows - 1) / kTileRows;
    TileIter it(T, remap, walkers ? walkers : gridDim.x);
    if (!it.valid()) return;
    // pf = 1: the row pointers of the next tile are loaded while the current
    // tile's entries stream in, so each tile starts with its bounds at hand.
    TileMeta<P> cur, nxt;
    cur.load(rp, n, it.tile());
    while (true) {
        TileIter after = it;
        after.next();
        const bool more = after.valid();
        const int64_t r1 = min(cur.r0 + static_cast<int64_t>(kTileRows), n);
        const int64_t row = cur.r0 + threadIdx.x;
        const int64_t s = cur.first(), e = cur.end();
        const int64_t a = cur.lo(), b = cur.hi();
        const bool lng = LR && row < r1 && b - a > kLongRow;
        if (e - s <= kStreamCap) {
            dma_chunks<V>(va, s, e, nnz, lv, nt);
            dma_chunks<I>(ci, s, e, nnz, lc, nt);
            if (more && pf) nxt.load(rp, n, after.tile());
            const auto pv = pre_of(epi, row < r1 ? row : r1 - 1);   // every lane loads
            __builtin_amdgcn_s_waitcnt(0);   // this wave's DMA (and the prefetches) has landed
            __syncthreads();                 // ... and every other wave's
            // The row sums run at raised wave priority, so on a SIMD shared
            // with workgroups that are issuing or awaiting their next tile's
            // DMA they finish first and free their LDS sooner.
            __builtin_amdgcn_s_setprio(2);
            const int64_t s0v = s & ~static_cast<int64_t>(Chunks<V>::EPC - 1);
            const int64_t s0c = s & ~static_cast<int64_t>(Chunks<I>::EPC - 1);
            if (row < r1 && !lng) emit_row(epi, row, row_from_lds<V, I, C>(sv, sc, a, b, s0v, s0c, gx, col, row), pv);
            __builtin_amdgcn_s_setprio(0);
            lds_barrier();                   // LDS free for the next tile (the row's stores stay in flight)
        } else {
            if (more && pf) nxt.load(rp, n, after.tile());
            const auto pv = pre_of(epi, row < r1 ? row : r1 - 1);
            if (row < r1 && !lng) emit_row(epi, row, row_from_global<V, I, C>(va, ci, a, b, gx, nt, col, row), pv);
        }
        if constexpr (LR)
            long_rows<C>(lng, rp, n, cur.r0, gx, col, epi, [&](int64_t k) { return ldv(va + k, nt); },
                         [&](int64_t k) { return ci[k]; });
        if (!more) break;
        if (!pf) nxt.load(rp, n, after.tile());
        it = after;
        cur = nxt;
    }
}

// The gather of the product's input vector: x[c] itself, unless the epilogue
// forms the vector on the fly (it then provides gather(), e.g. the fused CG
// step, whose direction p_k = r_{k-1} - alpha q_{k-1} + beta p_{k-1} is
// formed at every gathered column).
template <class Epi, class = void>
struct HasGather : std::false_type {};
template <class Epi>
struct HasGather<Epi, std::void_t<decltype(std::declval<const Epi &>().gather())>> : std::true_type {};

template <typename X, typename C, class Epi>
__device__ __forceinline__ auto gather_of(const Epi &epi, const X *x) {
    if constexpr (HasGather<Epi>::value) return epi.gather();
    else return PlainGather<X, C>{x};
}

// Register budget of the row-tile kernel, as waves per SIMD it must fit: the
// CG loop's product on coded FP64 tiles with packed rows (an epilogue that
// declares kHotLoop) is held to seven, where it otherwise lands one
// register above the budget and loses a workgroup per CU to it; every other
// instance is left to the compiler.
template <class Epi, class = void>
struct HotLoop : std::false_type {};
template <class Epi>
struct HotLoop<Epi, std::void_t<decltype(Epi::kHotLoop)>> : std::bool_constant<Epi::kHotLoop> {};

template <typename V, typename P, class Epi>
constexpr int spmv_min_waves() {
    return std::is_same_v<V, double> && std::is_same_v<P, RowPack> && HotLoop<Epi>::value ? 7 : 1;
}

// walkers: the workgroups that walk the tiles (0 = all).  A grid sized for
// the autotuned kernel can exceed what another epilogue's kernel holds
// resident; the workgroups past the resident count would then start only
// when the first ones finish and walk their tiles alone.  They take no
// tiles instead and store zero partials, so a consumer still sums one
// partial per launched workgroup and gets the same total.
template <typename V, typename P, typename I, typename X, typename C, class Epi, bool LR = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(spmv_min_waves<V, P, Epi>()))) void k_spmv_stream(int64_t n, int64_t nnz, const P *__restrict__ rp,
                                                        const I *__restrict__ ci, const V *__restrict__ va,
                                                        const X *__restrict__ x, int remap, int nt, int pf,
                                                        int walkers, Epi epi_in) {
    Epi epi = epi_in;
    if (epi.skip()) return;
    const uint32_t W = walkers > 0 && static_cast<uint32_t>(walkers) < gridDim.x ? walkers : gridDim.x;
    if (blockIdx.x >= W) {   // uniform
        epi.finish();
        return;
    }
    __shared__ u32x4 lv[Chunks<V>::LDS];
    __shared__ u32x4 lc[Chunks<I>::LDS];
    if constexpr (std::is_same_v<I, Code8>) {
        // the offset table sits in the kCodeDict * 8 bytes before the codes
        __shared__ int64_t dict[kCodeDict];
        const int64_t *g = reinterpret_cast<const int64_t *>(ci) - kCodeDict;
        for (int i = threadIdx.x; i < kCodeDict; i += kBlock) dict[i] = g[i];
        __syncthreads();
        spmv_tiles_lds<V, P, I, C, LR>(n, nnz, rp, ci, va, gather_of<X, C>(epi, x), remap, nt, pf, epi, lv, lc,
                                       ColCoded{dict}, W);
    } else {
        spmv_tiles_lds<V, P, I, C, LR>(n, nnz, rp, ci, va, gather_of<X, C>(epi, x), remap, nt, pf, epi, lv, lc,
                                       ColPlain{}, W);
    }
    epi.finish();
}

template <typename V, typename P, typename I, typename C, class Gx, class Epi>
__device__ __forceinline__ void spmv_tiles_vector(int64_t n, const P *__restrict__ rp, const I *__restrict__ ci,
                                                  const V *__restrict__ va, const Gx &gx, int lanes_log2, int remap,
                                                  int nt, Epi &epi) {
    const int L = 1 << lanes_log2;
    const int lane = threadIdx.x & (L - 1);
    const int group = threadIdx.x >> lanes_log2;
    const int groups = kBlock >> lanes_log2;
    const int64_t T = (n + kTileRows - 1) / kTileRows;
    for (TileIter it(T, remap); it.valid(); it.next()) {
        const int64_t r0 = it.tile() * kTileRows;
        const int64_t r1 = min(r0 + (int64_t)kTileRows, n);
        for (int pass = 0; pass < L; ++pass) {
            const int64_t row = r0 + static_cast<int64_t>(pass) * groups + group;
            C sum = 0;
            if (row < r1) {
                const int64_t a = static_cast<int64_t>(rp[row]), b = static_cast<int64_t>(rp[row + 1]);
                for (int64_t k = a + lane; k < b; k += L)
                    sum = fma(static_cast<C>(widen(ldv(va + k, nt))), static_cast<C>(gx(static_cast<int64_t>(ci[k]))),
                              sum);
            }
            for (int off = L >> 1; off >= 1; off >>= 1) sum += __shfl_xor(sum, off, 64);
            if (row < r1 && lane == 0) epi.row(row, sum);
        }
    }
}

template <typename V, typename P, typename I, typename X, typename C, class Epi>
__global__ __launch_bounds__(kBlock) void k_spmv_vector(int64_t n, const P *__restrict__ rp,
                                                        const I *__restrict__ ci, const V *__restrict__ va,
                                                        const X *__restrict__ x, int lanes_log2, int remap,
                                                        int nt, Epi epi_in) {
    Epi epi = epi_in;
    if (epi.skip()) return;
    spmv_tiles_vector<V, P, I, C>(n, rp, ci, va, gather_of<X, C>(epi, x), lanes_log2, remap, nt, epi);
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

// Workgroups of kernel Kern resident on one CU at once (asked once per
// kernel; 0 if the runtime cannot tell).
template <auto Kern>
int resident_per_cu() {
    static const int blocks = [] {
        int b = 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, Kern, kBlock, 0) == hipSuccess ? b : 0;
    }();
    return blocks;
}

template <typename V, typename X, typename C, class Epi>
hipError_t launch_family(const CsrDev &A, const SpmvTune &t, const X *x, const Epi &epi, hipStream_t s) {
    if (A.n_rows == 0) return hipSuccess;
    // tile walkers of a row-tile kernel: the grid, or as many workgroups as
    // that kernel holds resident on the device if fewer
    auto walkers = [&](int per_cu) { return t.cus > 0 && per_cu > 0 ? std::min(t.grid, t.cus * per_cu) : 0; };
    return dispatch_idx(A, [&](auto rp, auto ci) {
        using P = pointee_t<decltype(rp)>;
        using I = pointee_t<decltype(ci)>;
        const V *va = static_cast<const V *>(A.va);
        const dim3 grid(t.grid), block(kBlock);
        // the LDS tiles DMA the values (and the plain column indices) in
        // 16-byte chunks; arrays without that alignment take one lane per
        // row, which sums each row in the same order
        auto al16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
        // column codes exist only for matrices without rows longer than
        // kLongRow (the plan's rule), so only the plain-index kernel has a
        // long-row instance
        const bool coded = t.kind == 0 && t.codes && A.codes;
        const bool lr = A.max_row > kLongRow;
        if (t.kind == 0 && !(al16(A.va) && (coded || al16(A.ci)))) {
            hipLaunchKernelGGL((k_spmv_vector<V, P, I, X, C, Epi>), grid, block, 0, s, A.n_rows, rp, ci, va, x, 0,
                               t.xcd_remap, t.nt, epi);
        } else if (coded && t.pack && A.rowpack) {
            constexpr auto K = k_spmv_stream<V, RowPack, Code8, X, C, Epi>;
            hipLaunchKernelGGL(K, grid, block, 0, s, A.n_rows, A.nnz, static_cast<const RowPack *>(A.rowpack),
                               static_cast<const Code8 *>(A.codes), va, x, t.xcd_remap, t.nt, t.pf, walkers(resident_per_cu<K>()), epi);
        } else if (coded) {
            constexpr auto K = k_spmv_stream<V, P, Code8, X, C, Epi>;
            hipLaunchKernelGGL(K, grid, block, 0, s, A.n_rows, A.nnz, rp, static_cast<const Code8 *>(A.codes), va, x,
                               t.xcd_remap, t.nt, t.pf, walkers(resident_per_cu<K>()), epi);
        } else if (t.kind == 0 && lr) {
            constexpr auto K = k_spmv_stream<V, P, I, X, C, Epi, true>;
            hipLaunchKernelGGL(K, grid, block, 0, s, A.n_rows, A.nnz, rp, ci, va, x, t.xcd_remap, t.nt, t.pf,
                               walkers(resident_per_cu<K>()), epi);
        } else if (t.kind == 0) {
            constexpr auto K = k_spmv_stream<V, P, I, X, C, Epi>;
            hipLaunchKernelGGL(K, grid, block, 0, s, A.n_rows, A.nnz, rp, ci, va, x, t.xcd_remap, t.nt, t.pf,
                               walkers(resident_per_cu<K>()), epi);
        } else {
            hipLaunchKernelGGL((k_spmv_vector<V, P, I, X, C, Epi>), grid, block, 0, s, A.n_rows, rp, ci, va, x,
                               t.lanes_log2, t.xcd_remap, t.nt, epi);
        }
        return hipGetLastError();
    });
}

}  // namespace tile
}  // namespace spk
