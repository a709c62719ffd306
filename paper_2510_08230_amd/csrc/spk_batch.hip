// Batched serving kernels: every live slot (one solve request) advances by one
// step of its phase per tick, all slots in the same six launches.
//
// A mixed request is solved by FP32 CG (FP64 dot products) with FP64
// iterative refinement, exactly as the single-solve mixed path does; an
// FP64 request runs the same phases with an FP64 inner CG whose stop test
// is the final one (||r|| <= tau ||b||), so with x0 = 0 it is plain CG and
// the outer step only confirms the true residual.  Both run on per-slot
// 256-row tiles: the launch walks a global tile list (slot, local tile), and
// every per-slot reduction is over per-TILE partials summed in a fixed order
// by one workgroup per slot.  Tile boundaries and reduction trees depend only
// on the request's own n, so a request's result is bitwise the same alone and
// in any mix of other requests.
//
// Phases: OUTER (r = b - A x in FP64; r32 = p32 = fl32(r), d = 0) ->
// INNER (CG on A32 d = r32 until ||r_in|| <= tau_in ||r32||; FP64 requests:
// CG on A d = r until ||r_in|| <= tau ||b||) -> CORRECT
// (x += d) -> OUTER ... -> DONE when ||b - A x|| <= tau ||b|| (or a cap).
// Scalars a launch writes are read only by later launches; the phase a tick
// acts on is committed by the last launch of the tick.
#include "spk_device.h"
#include "spk_launch.h"

namespace spk {
namespace {

using namespace dev;

// Row sum of this thread's row of the 256-row tile [r0, r1) (int32 indices),
// values and columns staged in LDS by DMA.  has_row: this thread owns a row.
// stage = 0 (arrays not 16-byte aligned): rows read values and columns directly.
template <typename V, typename X, typename C>
__device__ __forceinline__ C tile_row_sum(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                          const V *__restrict__ va, int64_t nnz, const X *__restrict__ x, int64_t r0,
                                          int64_t r1, u32x4 *lv, u32x4 *lc, bool &has_row, int stage, int nt) {
    const int64_t s = rp[r0], e = rp[r1];
    const int64_t row = r0 + threadIdx.x;
    int64_t a = 0, b = 0;
    has_row = row < r1;
    if (has_row) {
        a = rp[row];
        b = rp[row + 1];
    }
    C sum = 0;
    if (stage && e - s <= kStreamCap) {
        dma_chunks<V>(va, s, e, nnz, lv, nt);
        dma_chunks<int32_t>(ci, s, e, nnz, lc, nt);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        __builtin_amdgcn_s_setprio(2);   // row sums ahead of other workgroups' DMA issue
        if (has_row)
            sum = row_from_lds<V, int32_t, C>(reinterpret_cast<const V *>(lv), reinterpret_cast<const int32_t *>(lc), a,
                                              b, s & ~static_cast<int64_t>(Chunks<V>::EPC - 1),
                                              s & ~static_cast<int64_t>(Chunks<int32_t>::EPC - 1),
                                              PlainGather<X, C>{x});
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
    } else if (has_row) {
        sum = row_from_global<V, int32_t, C>(va, ci, a, b, PlainGather<X, C>{x}, nt);
    }
    return sum;
}

__global__ __launch_bounds__(kBlock) void k_b_spmv(BatchDev B) {
    __shared__ u32x4 lv[Chunks<double>::LDS];
    __shared__ u32x4 lc[Chunks<int32_t>::LDS];
    for (TileIter it(B.counts[0], B.remap); it.valid(); it.next()) {
        const int2 te = B.tiles[it.tile()];
        const SlotDesc &D = B.desc[te.x];
        const SlotState &S = B.state[te.x];
        const int ph = S.phase;
        const int64_t r0 = static_cast<int64_t>(te.y) * kTileRows;
        const int64_t r1 = min(r0 + static_cast<int64_t>(kTileRows), D.n);
        const int64_t row = r0 + threadIdx.x;
        bool has = false;
        const bool inner = ph == PH_INNER && S.stop_in == STOP_RUNNING;
        if (inner && !D.fp64) {
            const float s = tile_row_sum<float, float, float>(D.rp, D.ci, D.va32, D.nnz, D.p, r0, r1, lv, lc, has, D.stage,
                                                              B.nt);
            double v[1] = {0.0};
            if (has) {
                D.q[row] = s;
                v[0] = static_cast<double>(D.p[row]) * static_cast<double>(s);
            }
            block_reduce_store<1>(v, D.part + PART_PQ * D.tiles + te.y, D.tiles);
        } else if (inner || ph == PH_OUTER) {
            // FP64 products: an FP64 request's q = A p, or any request's A x
            const double s = tile_row_sum<double, double, double>(D.rp, D.ci, D.va64, D.nnz, inner ? D.p64 : D.x, r0,
                                                                  r1, lv, lc, has, D.stage, B.nt);
            if (inner) {
                double v[1] = {0.0};
                if (has) {
                    D.q64[row] = s;
                    v[0] = D.p64[row] * s;
                }
                block_reduce_store<1>(v, D.part + PART_PQ * D.tiles + te.y, D.tiles);
            } else {
                double v[3] = {0.0, 0.0, 0.0};
                if (has) {
                    const double bi = D.b[row];
                    const double ri = bi - s;
                    if (D.fp64) {
                        D.r64[row] = ri;
                        D.p64[row] = ri;
                        D.d64[row] = 0.0;
                        v[1] = ri * ri;
                    } else {
                        const float r32 = static_cast<float>(ri);
                        D.r[row] = r32;
                        D.p[row] = r32;
                        D.d[row] = 0.0f;
                        v[1] = static_cast<double>(r32) * static_cast<double>(r32);
                    }
                    v[0] = ri * ri;
                    v[2] = bi * bi;
                }
                block_reduce_store<3>(v, D.part + PART_OUT * D.tiles + te.y, D.tiles);
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_b_reduce_a(BatchDev B) {
    const int NS = B.counts[1];
    for (int j = blockIdx.x; j < NS; j += gridDim.x) {
        const int sl = B.slots[j];
        const SlotDesc &D = B.desc[sl];
        SlotState &S = B.state[sl];
        const int ph = S.phase;
        if (ph == PH_INNER && S.stop_in == STOP_RUNNING) {
            double tot[1];
            sum_partials<1>(D.part + PART_PQ * D.tiles, D.tiles, D.tiles, tot);
            if (threadIdx.x == 0) {
                const double pq = tot[0];
                if (!isfinite(pq)) S.stop_in = STOP_NON_FINITE;
                else if (pq <= 0.0) S.stop_in = STOP_BREAKDOWN;
                else S.alpha = S.rho[S.iter_in & 3] / pq;
            }
        } else if (ph == PH_OUTER) {
            double tot[3];
            sum_partials<3>(D.part + PART_OUT * D.tiles, D.tiles, D.tiles, tot);
            if (threadIdx.x == 0) {
                const double rn = sqrt(tot[0]), bn = sqrt(tot[2]), r32 = sqrt(tot[1]);
                S.bnorm = bn;
                S.rnorm = rn;
                if (!isfinite(bn) || !isfinite(rn)) {
                    S.stop = STOP_NON_FINITE;
                    S.next_phase = PH_DONE;
                } else if (bn == 0.0) {
                    S.rnorm = 0.0;
                    S.stop = STOP_CONVERGED;
                    S.next_phase = PH_ZEROX;
                } else if (rn <= D.tau * bn) {
                    S.stop = STOP_CONVERGED;
                    S.next_phase = PH_DONE;
                } else if (S.outer >= D.max_outer || S.iters >= D.max_iters) {
                    S.stop = STOP_MAX_ITERS;
                    S.next_phase = PH_DONE;
                } else if (tot[1] == 0.0) {   // residual below FP32 range: no inner progress possible
                    S.stop = STOP_BREAKDOWN;
                    S.next_phase = PH_DONE;
                } else {
                    S.rho[0] = tot[1];
                    S.thresh_in = D.fp64 ? D.tau * bn : D.tau_in * r32;
                    S.iter_in = 0;
                    S.stop_in = STOP_RUNNING;
                    S.next_phase = PH_INNER;
                }
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_b_update(BatchDev B) {
    for (TileIter it(B.counts[0], B.remap); it.valid(); it.next()) {
        const int2 te = B.tiles[it.tile()];
        const SlotDesc &D = B.desc[te.x];
        const SlotState &S = B.state[te.x];
        const int ph = S.phase;
        const int64_t r0 = static_cast<int64_t>(te.y) * kTileRows;
        const int64_t row = r0 + threadIdx.x;
        const bool has = row < D.n;
        if (ph == PH_INNER && S.stop_in == STOP_RUNNING) {
            double v[1] = {0.0};
            if (has) {
                if (D.fp64) {
                    const double alpha = S.alpha;
                    D.d64[row] = fma(alpha, D.p64[row], D.d64[row]);
                    const double ri = fma(-alpha, D.q64[row], D.r64[row]);
                    D.r64[row] = ri;
                    v[0] = ri * ri;
                } else {
                    const float alpha = static_cast<float>(S.alpha);
                    D.d[row] = fmaf(alpha, D.p[row], D.d[row]);
                    const float ri = fmaf(-alpha, D.q[row], D.r[row]);
                    D.r[row] = ri;
                    v[0] = static_cast<double>(ri) * static_cast<double>(ri);
                }
            }
            block_reduce_store<1>(v, D.part + PART_RR * D.tiles + te.y, D.tiles);
        } else if (ph == PH_CORRECT) {
            if (has) D.x[row] += D.fp64 ? D.d64[row] : static_cast<double>(D.d[row]);
        } else if (ph == PH_ZEROX) {
            if (has) D.x[row] = 0.0;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_b_reduce_b(BatchDev B) {
    const int NS = B.counts[1];
    for (int j = blockIdx.x; j < NS; j += gridDim.x) {
        const int sl = B.slots[j];
        const SlotDesc &D = B.desc[sl];
        SlotState &S = B.state[sl];
        const int ph = S.phase;
        if (ph == PH_INNER) {
            if (S.stop_in == STOP_RUNNING) {
                double tot[1];
                sum_partials<1>(D.part + PART_RR * D.tiles, D.tiles, D.tiles, tot);
                if (threadIdx.x == 0) {
                    const int64_t k = S.iter_in, k1 = k + 1;
                    const double rho_new = tot[0];
                    const double res = sqrt(rho_new);
                    S.iter_in = k1;
                    S.iters += 1;
                    if (!isfinite(rho_new)) S.stop_in = STOP_NON_FINITE;
                    else if (res <= S.thresh_in) S.stop_in = STOP_CONVERGED;
                    else if (S.iters >= D.max_iters) S.stop_in = STOP_MAX_ITERS;
                    else {
                        S.beta = rho_new / S.rho[k & 3];
                        S.rho[k1 & 3] = rho_new;
                    }
                }
            }
            if (threadIdx.x == 0 && S.stop_in != STOP_RUNNING) {
                if ((S.stop_in == STOP_BREAKDOWN || S.stop_in == STOP_NON_FINITE) && S.iter_in == 0) {
                    S.stop = S.stop_in;
                    S.next_phase = PH_DONE;
                } else {
                    S.next_phase = PH_CORRECT;
                }
            }
        } else if (ph == PH_CORRECT) {
            if (threadIdx.x == 0) {
                S.outer += 1;
                S.next_phase = PH_OUTER;
            }
        } else if (ph == PH_ZEROX) {
            if (threadIdx.x == 0) S.next_phase = PH_DONE;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_b_pupdate(BatchDev B) {
    for (TileIter it(B.counts[0], B.remap); it.valid(); it.next()) {
        const int2 te = B.tiles[it.tile()];
        const SlotDesc &D = B.desc[te.x];
        const SlotState &S = B.state[te.x];
        if (S.phase != PH_INNER || S.stop_in != STOP_RUNNING) continue;
        const int64_t row = static_cast<int64_t>(te.y) * kTileRows + threadIdx.x;
        if (row >= D.n) continue;
        if (D.fp64) D.p64[row] = fma(S.beta, D.p64[row], D.r64[row]);
        else D.p[row] = fmaf(static_cast<float>(S.beta), D.p[row], D.r[row]);
    }
}

__global__ __launch_bounds__(kBlock) void k_b_commit(BatchDev B) {
    const int NS = B.counts[1];
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < NS; j += gridDim.x * kBlock) {
        const int sl = B.slots[j];
        SlotState &S = B.state[sl];
        S.phase = S.next_phase;
        SlotStatus &st = B.status[sl];
        st.phase = S.phase;
        st.stop = S.stop;
        st.iters = S.iters;
        st.outer = S.outer;
        st.rnorm = S.rnorm;
        st.bnorm = S.bnorm;
    }
}

__global__ __launch_bounds__(kBlock) void k_round_f32(int64_t nnz, const double *__restrict__ src,
                                                      float *__restrict__ dst) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < nnz; i += stride)
        dst[i] = static_cast<float>(src[i]);
}

// dst[i] = src[i] for 64-bit indices known to fit 32 bits (a validated
// request's row pointers or columns, below 2^31).
__global__ __launch_bounds__(kBlock) void k_narrow_i32(int64_t count, const int64_t *__restrict__ src,
                                                       int32_t *__restrict__ dst) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < count; i += stride)
        dst[i] = static_cast<int32_t>(src[i]);
}

}  // namespace

hipError_t launch_narrow_i32(int64_t count, const int64_t *src, int32_t *dst, int grid, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_narrow_i32, dim3(grid), dim3(kBlock), 0, s, count, src, dst);
    return hipGetLastError();
}

hipError_t launch_batch_tick(const BatchDev &B, hipStream_t s) {
    hipLaunchKernelGGL(k_b_spmv, dim3(B.tile_grid), dim3(kBlock), 0, s, B);
    hipLaunchKernelGGL(k_b_reduce_a, dim3(B.slot_grid), dim3(kBlock), 0, s, B);
    hipLaunchKernelGGL(k_b_update, dim3(B.tile_grid), dim3(kBlock), 0, s, B);
    hipLaunchKernelGGL(k_b_reduce_b, dim3(B.slot_grid), dim3(kBlock), 0, s, B);
    hipLaunchKernelGGL(k_b_pupdate, dim3(B.tile_grid), dim3(kBlock), 0, s, B);
    hipLaunchKernelGGL(k_b_commit, dim3(1), dim3(kBlock), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_round_f32(int64_t nnz, const double *src, float *dst, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_round_f32, dim3(grid), dim3(kBlock), 0, s, nnz, src, dst);
    return hipGetLastError();
}

int batch_tile_blocks_per_cu() {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_b_spmv, kBlock, 0) != hipSuccess || blocks < 1) blocks = 1;
    return blocks;
}

}  // namespace spk
