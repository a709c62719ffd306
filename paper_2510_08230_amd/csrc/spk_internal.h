// Internal declarations shared by the host runtime (spk_api.cpp) and the
// gfx950 kernels (spk_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace spk {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64s)
constexpr int kTileRows = 256;     // rows per SpMV tile
constexpr int kMaxGrid = 8192;     // cap on workgroups of any grid-stride launch
constexpr int kNumXcd = 8;         // MI355X: 8 XCDs, workgroups dispatched round-robin

enum Stop : int32_t {
    STOP_RUNNING = 0,
    STOP_CONVERGED = 1,
    STOP_MAX_ITERS = 2,
    STOP_BREAKDOWN = 3,
    STOP_NON_FINITE = 4
};

// Reduction sites: each owns an arrival counter and a partials slab.
enum Site : int { SITE_INIT = 0, SITE_PQ = 1, SITE_RR = 2, SITE_TRUE = 3, SITE_COUNT = 4 };
constexpr int kSiteWidth = 2;      // values reduced at once per site (max)

// Device-resident scalars of one CG solve.  Loop kernels read only fields
// written by earlier launches; workgroup 0 of a launch writes the results.
struct SolveState {
    double rho[4];        // ring: rho[k & 3] = r_k . r_k
    double pq, alpha;     // last p.q and alpha (diagnostics)
    double bnorm;         // ||b||
    double thresh;        // reduction_factor * ||b||
    double resnorm;       // sqrt(rho) at the last check
    double true_resnorm;  // ||b - A x|| at exit (NaN if not computed)
    int64_t base;         // absolute index of the current chunk's first iteration
    int64_t iter;         // completed updates
    int64_t max_iters;
    int32_t stop;         // Stop
    int32_t zero_x;       // b == 0: the finaliser sets x = 0
    double *x;            // caller's solution vector for this execute
    double *hist;         // optional ||r_k|| history
    int64_t hist_cap;
};

// Launch shape of the SpMV family (shared by every SpMV-based kernel).
struct SpmvTune {
    int kind;        // 0 = LDS-staged row tiles, 1 = lanes-per-row vector kernel
    int lanes_log2;  // vector kernel: log2(lanes per row)
    int grid;        // workgroups
    int xcd_remap;   // 1 = contiguous tile ranges per XCD
    int nt;          // 1 = non-temporal loads for the matrix value stream
    int pf;          // LDS tiles: 1 = next tile's loads issued before the current tile is reduced
    int bpc;         // workgroups per CU the grid was sized for
};

// Device CSR view with runtime-typed arrays.
struct CsrDev {
    int64_t n_rows, n_cols, nnz;
    int ptr_t, idx_t, val_t;   // spk_itype / spk_dtype codes
    const void *rp, *ci, *va;
};

// Validation flag bits (set by the GPU check, order resolved on the host).
enum : unsigned { VFLAG_BAD_FIRST = 1u, VFLAG_DECREASING = 2u, VFLAG_BAD_LAST = 4u, VFLAG_BAD_COLUMN = 8u };

// ---- launchers (spk_kernels.hip) -------------------------------------------------
hipError_t launch_validate(const CsrDev &A, unsigned *flags, int max_grid, hipStream_t s);
hipError_t launch_partition(const CsrDev &A, int64_t parts, int64_t *split, hipStream_t s);

// y = A x; x/y are double for F64 values, float otherwise.
hipError_t launch_spmv(const CsrDev &A, const SpmvTune &t, const void *x, void *y, hipStream_t s);

// CG (FP64).  partials: SITE_COUNT * kSiteWidth * kMaxGrid doubles.
// Iteration j of a chunk = spmv_pq, update(j), pupdate(j); a chunk of c
// iterations ends with chunk_end(c).
hipError_t launch_cg_init(const CsrDev &A, const SpmvTune &t, const double *b, double *x, double *r,
                          double *p, SolveState *st, double *partials, double tau, int64_t max_iters,
                          double *hist, int64_t hist_cap, hipStream_t s);
hipError_t launch_cg_spmv_pq(const CsrDev &A, const SpmvTune &t, const double *p, double *q,
                             SolveState *st, double *partials, hipStream_t s);
hipError_t launch_cg_update(int64_t n, int grid, int spmv_grid, int j, const double *p, double *r,
                            const double *q, SolveState *st, double *partials, hipStream_t s);
hipError_t launch_cg_pupdate(int64_t n, int grid, int j, const double *r, double *p, SolveState *st,
                             double *partials, hipStream_t s);
hipError_t launch_cg_chunk_end(SolveState *st, int count, hipStream_t s);
// Sets x = 0 when b == 0, then (optionally) recomputes ||b - A x|| into the state.
hipError_t launch_cg_finalize(const CsrDev &A, const SpmvTune &t, const double *b, double *x,
                              SolveState *st, double *partials, int true_residual, hipStream_t s);

hipError_t launch_copy(const void *src, void *dst, size_t bytes, int grid, hipStream_t s);

// Workgroups of the SpMV kernel resident per CU for this tune/type (occupancy API).
int spmv_blocks_per_cu(const CsrDev &A, const SpmvTune &t);

}  // namespace spk
