// Device helpers shared by the gfx950 kernel translation units: value
// widening, fixed-order reductions, the LDS-DMA tile staging of CSR values and
// column indices, and the per-row reducers.  Everything here is internal
// linkage (header-only, inline/static).
#pragma once

#include "spk_internal.h"

#include <cmath>
#include <type_traits>

namespace spk {
namespace dev {

struct bf16s { uint16_t bits; };

__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ float widen(_Float16 v) { return static_cast<float>(v); }
__device__ __forceinline__ float widen(bf16s v) { return __uint_as_float(static_cast<unsigned>(v.bits) << 16); }

// Matrix-value load, optionally non-temporal (streamed data that should not
// displace the gathered vector from the caches).
template <typename T>
__device__ __forceinline__ T ldv(const T *p, int nt) {
    return nt ? __builtin_nontemporal_load(p) : *p;
}
__device__ __forceinline__ bf16s ldv(const bf16s *p, int nt) {
    bf16s r;
    r.bits = nt ? __builtin_nontemporal_load(&p->bits) : p->bits;
    return r;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Tiles visited by this workgroup (workgroups are dispatched round-robin over
// the 8 XCDs, workgroup b on XCD b % 8).
//   remap = 0: tile t -> workgroup t mod G (consecutive tiles on different XCDs)
//   remap = 1: XCD x walks the contiguous eighth [x T/8, (x+1) T/8)
//   remap = k >= 2: tiles grouped in blocks of k; block B belongs to XCD B % 8,
//     and each XCD walks its blocks in order, so all XCDs sweep one front
//     while each block's neighbouring rows share one L2.
// Every tile loop copies the iterator once per tile, so it is kept to a few
// 32-bit words (tile counts stay below 2^31): a wider iterator measured 43%
// slower on the FP32 products.  Block sizes that are powers of two (the
// autotuner's 64 and 256) step by shifts.
struct TileIter {
    uint32_t j, end, stride;   // position in this XCD's (or the global) tile sequence
    uint32_t k, xcd;           // block size and XCD (remap >= 2)
    int shift;                 // log2 k when k is a power of two, else -1
    int mode;
    __device__ TileIter(int64_t T64, int remap) : TileIter(T64, remap, gridDim.x) {}
    // G: the workgroups that walk the tiles (the first G of the grid)
    __device__ TileIter(int64_t T64, int remap, uint32_t G) {
        const uint32_t b = blockIdx.x, T = static_cast<uint32_t>(T64);
        mode = (G >= kNumXcd && remap >= 1) ? (remap == 1 ? 1 : 2) : 0;
        k = remap >= 2 ? static_cast<uint32_t>(remap) : 1u;
        shift = (k & (k - 1)) == 0 ? __builtin_ctz(k) : -1;
        xcd = b % kNumXcd;
        const uint32_t m = b / kNumXcd;
        const uint32_t M = (G - xcd + kNumXcd - 1) / kNumXcd;   // workgroups on this XCD
        if (mode == 0) {
            j = b;
            end = T;
            stride = G;
        } else if (mode == 1) {
            j = static_cast<uint32_t>((static_cast<uint64_t>(xcd) * T) / kNumXcd) + m;
            end = static_cast<uint32_t>((static_cast<uint64_t>(xcd + 1) * T) / kNumXcd);
            stride = M;
        } else {
            // tiles of this XCD: blocks xcd, xcd + 8, ...; the last block may be short
            const uint32_t nb = (T + k - 1) / k;                    // blocks
            const uint32_t my_blocks = nb > xcd ? (nb - xcd + kNumXcd - 1) / kNumXcd : 0;
            uint32_t count = my_blocks * k;
            if (my_blocks > 0 && (xcd + (my_blocks - 1) * kNumXcd) == nb - 1) count -= nb * k - T;
            j = m;
            end = count;
            stride = M;
        }
    }
    __device__ bool valid() const { return j < end; }
    __device__ void next() { j += stride; }
    __device__ int64_t tile() const {
        if (mode != 2) return j;
        const uint32_t q = shift >= 0 ? (j >> shift) : j / k;
        const uint32_t r = j - q * k;
        return static_cast<int64_t>(q * kNumXcd + xcd) * k + r;
    }
};

// Packed row pointers (tag type of the row-pointer argument): per tile an
// int64 first entry, then per row a uint16 offset from it.
struct RowPack {};

// Bounds of one row tile: its first row, its entry range [first(), end())
// and this thread's row range [lo(), hi()) (empty past the last row).
// load() issues every load unconditionally (a thread past the tile's last
// row re-reads that row's bounds) and keeps the loaded values as stored, so
// a load for the next tile stays in flight until the bounds are used: a
// load under a branch, or a value combined right after its load, is waited
// for at once.
template <typename P>
struct TileMeta {
    int64_t r0;
    P s, e, a, b;
    bool has;
    __device__ __forceinline__ void load(const P *__restrict__ rp, int64_t n, int64_t tile) {
        r0 = tile * kTileRows;
        const int64_t r1 = r0 + kTileRows < n ? r0 + kTileRows : n;
        s = rp[r0];
        e = rp[r1];
        const int64_t row = r0 + threadIdx.x;
        has = row < r1;
        const int64_t rr = has ? row : r1 - 1;
        a = rp[rr];
        b = rp[rr + 1];
    }
    __device__ __forceinline__ int64_t first() const { return static_cast<int64_t>(s); }
    __device__ __forceinline__ int64_t end() const { return static_cast<int64_t>(e); }
    __device__ __forceinline__ int64_t lo() const { return has ? static_cast<int64_t>(a) : 0; }
    __device__ __forceinline__ int64_t hi() const { return has ? static_cast<int64_t>(b) : 0; }
};

template <>
struct TileMeta<RowPack> {
    int64_t r0, s, e;
    uint16_t ra, rb;
    bool has, tail;   // tail: this thread's row is the tile's last (its end is e)
    __device__ __forceinline__ void load(const RowPack *__restrict__ rp, int64_t n, int64_t tile) {
        const int64_t *tb = reinterpret_cast<const int64_t *>(rp);
        const uint16_t *ro = reinterpret_cast<const uint16_t *>(tb + (n + kTileRows - 1) / kTileRows + 1);
        r0 = tile * kTileRows;
        const int64_t r1 = r0 + kTileRows < n ? r0 + kTileRows : n;
        s = tb[tile];
        e = tb[tile + 1];
        const int64_t row = r0 + threadIdx.x;
        has = row < r1;
        const int64_t rr = has ? row : r1 - 1;
        tail = rr + 1 >= r1;
        ra = ro[rr];
        rb = ro[tail ? rr : rr + 1];
    }
    __device__ __forceinline__ int64_t first() const { return s; }
    __device__ __forceinline__ int64_t end() const { return e; }
    __device__ __forceinline__ int64_t lo() const { return has ? s + ra : 0; }
    __device__ __forceinline__ int64_t hi() const { return has ? (tail ? e : s + rb) : 0; }
};

// Workgroup barrier for LDS only: LDS writes before it are seen by LDS
// reads after it, and global loads and stores still in flight stay in
// flight (__syncthreads also waits for those: a tile's result stores or the
// next tile's prefetched loads would then be drained at every tile).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block-level fixed-order reduction of NV doubles; thread 0 stores the
// workgroup's partials at partials[j * kMaxGrid + blockIdx.x].
template <int NV>
__device__ __forceinline__ void block_partial(double (&v)[NV], double *partials) {
    __shared__ double sh[NV][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double t = wave_sum(v[j]);
        if (lane == 0) sh[j][wid] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double t = sh[j][0];
#pragma unroll
            for (int w = 1; w < kBlock / 64; ++w) t += sh[j][w];
            partials[static_cast<size_t>(j) * kMaxGrid + blockIdx.x] = t;
        }
    }
}

// Every thread of the calling workgroup receives the fixed-order sums of the
// G partials partials[j * stride + b] (b < G) a previous launch stored
// (identical in every workgroup that calls it).  Each thread adds its
// strided share b = tid, tid + kBlock, ... in increasing b; the loads of up
// to 8 / NV strides (for every j) are issued before any of them is added, so
// a thread waits for one round trip per batch rather than per partial.
// Strides past G load a valid partial (the batch's first) and are not added.
template <int NV>
__device__ __forceinline__ void sum_partials(const double *partials, int64_t G, int64_t stride, double (&tot)[NV]) {
    __shared__ double sh[NV][kBlock / 64];
    constexpr int U = NV >= 8 ? 1 : 8 / NV;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double t[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) t[j] = 0.0;
    for (int64_t b0 = threadIdx.x; b0 < G; b0 += static_cast<int64_t>(U) * kBlock) {
        double v[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t b = b0 + static_cast<int64_t>(u) * kBlock;
            const int64_t bc = b < G ? b : b0;
#pragma unroll
            for (int j = 0; j < NV; ++j) v[u][j] = partials[static_cast<size_t>(j) * stride + bc];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (b0 + static_cast<int64_t>(u) * kBlock < G) {
#pragma unroll
                for (int j = 0; j < NV; ++j) t[j] += v[u][j];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double w = wave_sum(t[j]);
        if (lane == 0) sh[j][wid] = w;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double t = sh[j][0];
#pragma unroll
        for (int w = 1; w < kBlock / 64; ++w) t += sh[j][w];
        tot[j] = t;
    }
    __syncthreads();
}

template <int NV>
__device__ __forceinline__ void sum_partials(const double *partials, int G, double (&tot)[NV]) {
    sum_partials<NV>(partials, static_cast<int64_t>(G), static_cast<int64_t>(kMaxGrid), tot);
}

// Fixed-order workgroup reduction of NV doubles; thread 0 stores total j at
// out[j * stride].  Safe to call repeatedly (trailing barrier).
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], double *out, int64_t stride) {
    __shared__ double sh[NV][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double t = wave_sum(v[j]);
        if (lane == 0) sh[j][wid] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double t = sh[j][0];
#pragma unroll
            for (int w = 1; w < kBlock / 64; ++w) t += sh[j][w];
            out[static_cast<size_t>(j) * stride] = t;
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------ SpMV tilings
constexpr int kStreamCap = 2048;   // nnz staged in LDS per tile
#ifndef SPK_ROW_UNROLL
#define SPK_ROW_UNROLL 4
#endif
constexpr int kRowUnroll = SPK_ROW_UNROLL;   // gathers in flight per row step

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The contiguous nnz range [s, e) of one tile is copied into LDS in 16-byte
// chunks by the gfx950 global-to-LDS DMA (global_load_lds_dwordx4): lane l of
// a wave writes LDS bytes [16 l, 16 l + 16) past the wave's base, so no VGPR
// holds staged data.  The range is widened down to a 16-byte boundary (s0);
// chunk c covers elements [s0 + c*EPC, s0 + (c+1)*EPC).  Only a chunk running
// past the end of the array (the matrix's last chunk) is copied element-wise.
template <typename T>
struct Chunks {
    static constexpr int EPC = 16 / sizeof(T);
    static constexpr int MAXC = (kStreamCap / EPC + 1 + kBlock - 1) / kBlock;   // chunk rounds per thread
    static constexpr int LDS = kStreamCap / EPC + 1;                              // chunks per tile
};

typedef __attribute__((address_space(3))) void lds_void;

// nt = 1: the loads carry the non-temporal policy (the matrix streams through
// once; the gathered vector should keep its place in L2).
template <typename T>
__device__ __forceinline__ void dma_chunks(const T *__restrict__ g, int64_t s, int64_t e, int64_t total, u32x4 *lds,
                                           int nt) {
    constexpr int EPC = Chunks<T>::EPC;
    const int64_t s0 = s & ~static_cast<int64_t>(EPC - 1);
    const int lane = threadIdx.x & 63;
    const int wbase = threadIdx.x & ~63;
#pragma unroll
    for (int u = 0; u < Chunks<T>::MAXC; ++u) {
        const int cbase = u * kBlock + wbase;                  // this wave's first chunk this round
        if (s0 + static_cast<int64_t>(cbase) * EPC >= e) break;   // wave-uniform
        const int64_t k = s0 + static_cast<int64_t>(cbase + lane) * EPC;
        if (k < e) {
            if (k + EPC <= total) {
                if (nt)
                    __builtin_amdgcn_global_load_lds(static_cast<const void *>(g + k),
                                                     (lds_void *)(lds + cbase), 16, 0, 2);
                else
                    __builtin_amdgcn_global_load_lds(static_cast<const void *>(g + k),
                                                     (lds_void *)(lds + cbase), 16, 0, 0);
            } else {
                T *dst = reinterpret_cast<T *>(lds + cbase + lane);
                for (int j = 0; j < EPC; ++j)
                    if (k + j < total) dst[j] = g[k + j];
            }
        }
    }
}

// Gathers of the SpMV's input vector at column c.
template <typename X, typename C>
struct PlainGather {   // x[c]
    const X *__restrict__ x;
    __device__ __forceinline__ C operator()(int64_t c) const { return static_cast<C>(x[c]); }
};

template <typename T>
struct PUpdateGather {   // p_k[c] = fma(beta, p_{k-1}[c], r_k[c]): the CG direction formed on the fly
    T beta;
    const T *__restrict__ p_old;
    const T *__restrict__ r;
    __device__ __forceinline__ T operator()(int64_t c) const { return fma(beta, p_old[c], r[c]); }
};

// Column of an entry from its stored index.  ColPlain: the column index
// itself.  ColCoded: the entry holds a one-byte code, and the column is its
// row plus the code's offset in the matrix's table (held in LDS).
enum class Code8 : uint8_t {};

struct ColPlain {
    template <typename I>
    __device__ __forceinline__ int64_t operator()(I v, int64_t) const {
        static_assert(std::is_integral_v<I>, "coded columns need ColCoded");
        return static_cast<int64_t>(v);
    }
};

struct ColCoded {
    const int64_t *dict;   // LDS copy of the offset table
    __device__ __forceinline__ int64_t operator()(Code8 v, int64_t row) const {
        return row + dict[static_cast<uint8_t>(v)];
    }
};

// Sum of row [a, b) with values/columns read from LDS (offsets s0v / s0c).
template <typename V, typename I, typename C, class Gx, class D = ColPlain>
__device__ __forceinline__ C row_from_lds(const V *sv, const I *sc, int64_t a, int64_t b, int64_t s0v, int64_t s0c,
                                          const Gx &gx, const D &col = D{}, int64_t row = 0) {
    C sum = 0;
    for (int64_t k0 = a; k0 < b; k0 += kRowUnroll) {
        C av[kRowUnroll], xv[kRowUnroll];
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            const int64_t k = k0 + u;
            if (k < b) {
                av[u] = static_cast<C>(widen(sv[k - s0v]));
                xv[u] = static_cast<C>(gx(col(sc[k - s0c], row)));
            } else {
                av[u] = 0;
                xv[u] = 0;
            }
        }
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) sum = fma(av[u], xv[u], sum);
    }
    return sum;
}

template <typename V, typename I, typename C, class Gx, class D = ColPlain>
__device__ __forceinline__ C row_from_global(const V *__restrict__ va, const I *__restrict__ ci, int64_t a, int64_t b,
                                             const Gx &gx, int nt, const D &col = D{}, int64_t row = 0) {
    C sum = 0;
    for (int64_t k = a; k < b; ++k)
        sum = fma(static_cast<C>(widen(ldv(va + k, nt))), static_cast<C>(gx(col(ci[k], row))), sum);
    return sum;
}

}  // namespace dev
}  // namespace spk
