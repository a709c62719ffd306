// Launchers of the gfx950 kernels (defined beside their kernels in
// spk_kernels.hip, spk_krylov.hip, spk_gmres.hip and spk_batch.hip), called
// by the host runtime.  Not part of the public ABI.
#pragma once

#include "spk_internal.h"

namespace spk {

// ---- launchers (spk_kernels.hip) -------------------------------------------------
// CSR checks: flags[0] |= VFLAG_* bits, flags[1] = max(flags[1], the longest
// row's entry count, clamped to 2^32 - 1); both words zero before the launch.
hipError_t launch_validate(const CsrDev &A, unsigned *flags, int max_grid, hipStream_t s);
hipError_t launch_partition(const CsrDev &A, int64_t parts, int64_t *split, hipStream_t s);
// The distinct column offsets c - i of every step-th row tile (and the last)
// collected into table (kCodeSlots slots); words[0] counts them, words[1] is
// set when there are more than kCodeDict.  A must be valid.
hipError_t launch_pattern_probe(const CsrDev &A, int step, long long *table, unsigned *words, int grid,
                                hipStream_t s);
// Column codes (plan time): collects the distinct column offsets c - i of
// every step-th row tile (and the last) into table (kCodeSlots int64 words),
// then, when there are at most kCodeDict of them, writes the ascending offset
// table into the first kCodeDict * 8 bytes of codes_base and one code byte
// per entry after it, then (codes usable) the packed row pointers.  words
// holds 4 unsigned; afterwards words[0] = distinct offsets collected;
// words[1] = 0: codes usable, bit 0: more than kCodeDict offsets, bit 1: an
// entry's offset was not collected (sampled collection incomplete);
// words[2] != 0: a row offset within its tile exceeds 65535 (no packing).
// codes_base holds code_buffer_bytes(n_rows, nnz) bytes.
hipError_t launch_code_build(const CsrDev &A, int step, long long *table, unsigned *words, void *codes_base,
                             int grid, hipStream_t s);
// COO (idx_t 0 = int32, 1 = int64): flags gets VFLAG_BAD_FIRST for a row
// index out of range, VFLAG_BAD_COLUMN, VFLAG_UNSORTED for a decreasing row.
hipError_t launch_coo_validate(int64_t n_rows, int64_t n_cols, int64_t nnz, const void *row, const void *col,
                               int idx_t, unsigned *flags, int max_grid, hipStream_t s);
// Row pointer (n_rows + 1 entries of ptr_t) of a valid row-sorted COO matrix.
hipError_t launch_coo_rowptr(int64_t n_rows, int64_t nnz, const void *row, int idx_t, void *rp, int ptr_t,
                             hipStream_t s);

// y = A x; x/y are double for F64 values, float otherwise.
hipError_t launch_spmv(const CsrDev &A, const SpmvTune &t, const void *x, void *y, hipStream_t s);

// CG (FP64).  partials: SITE_COUNT * kSiteWidth * kMaxGrid doubles.
// Iteration j of a chunk = spmv_pq (q = A p, p.q partials), update(j)
// (alpha, r -= alpha q, r.r partials), pupdate(j) (x += alpha p, stop test,
// beta, p = r + beta p); a chunk of c iterations ends with chunk_end(c).
hipError_t launch_cg_init(const CsrDev &A, const SpmvTune &t, const double *b, double *x, double *r,
                          double *p, SolveState *st, double *partials, double tau, int64_t max_iters,
                          double *hist, int64_t hist_cap, hipStream_t s);
hipError_t launch_cg_spmv_pq(const CsrDev &A, const SpmvTune &t, const double *p, double *q,
                             SolveState *st, double *partials, hipStream_t s);
// Fused CG loop (one launch per iteration): the initial residual into
// f.r[1] with f.p[1] = f.q[1] = 0 (then the state as launch_cg_init), step j
// of a chunk (iteration st->base + j; x is the state's), and the FP32 inner
// step of the mixed solve (its x is the correction d); the refinement
// residual before a fused inner loop.
hipError_t launch_fcg_init(const CsrDev &A, const SpmvTune &t, const double *b, double *x, const FcgBufs<double> &f,
                           SolveState *st, double *partials, double tau, int64_t max_iters, double *hist,
                           int64_t hist_cap, hipStream_t s);
hipError_t launch_fcg_step(const CsrDev &A, const SpmvTune &t, int j, const FcgBufs<double> &f, SolveState *st,
                           double *partials, hipStream_t s);
hipError_t launch_fcg_step32(const CsrDev &A32, const SpmvTune &t, int j, const FcgBufs<float> &f, SolveState *st,
                             double *partials, hipStream_t s);
hipError_t launch_fcg_ir_residual(const CsrDev &A, const SpmvTune &t, const double *b, const double *x,
                                  const FcgBufs<float> &f, float *d32, SolveState *in, double *partials,
                                  double tau_in, int64_t max_inner, double *out, hipStream_t s);
hipError_t launch_cg_update(int64_t n, int grid, int spmv_grid, int j, double *r, const double *q, SolveState *st,
                            double *partials, hipStream_t s);
hipError_t launch_cg_pupdate(int64_t n, int grid, int j, const double *r, double *p, SolveState *st,
                             double *partials, hipStream_t s);
hipError_t launch_cg_chunk_end(SolveState *st, int count, hipStream_t s);

// Mixed precision: inner CG on FP32 vectors (A32 values F32, F16 or BF16),
// refinement steps in FP64 (A values F64, or F32 taken as exact).
hipError_t launch_cg_spmv_pq32(const CsrDev &A32, const SpmvTune &t, const float *p, float *q, SolveState *st,
                               double *partials, hipStream_t s);
hipError_t launch_cg_update32(int64_t n, int grid, int spmv_grid, int j, float *r, const float *q, SolveState *st,
                              double *partials, hipStream_t s);
hipError_t launch_cg_pupdate32(int64_t n, int grid, int j, const float *r, float *p, SolveState *st,
                               double *partials, hipStream_t s);
// r = b - A x (FP64); r32 = p32 = fl32(r), d32 = 0; inner state set up;
// out[0] = ||r||, out[1] = ||r32|| (device doubles).
hipError_t launch_ir_residual(const CsrDev &A, const SpmvTune &t, const double *b, const double *x, float *r32,
                              float *p32, float *d32, SolveState *in, double *partials, double tau_in,
                              int64_t max_inner, double *out, hipStream_t s);
hipError_t launch_ir_correct(int64_t n, int grid, double *x, const float *d, hipStream_t s);
// Round FP64 values to FP32 (bf16 = 0) or BF16 (bf16 = 1, round to nearest even).
// to: spk_dtype code 1 (F32), 2 (F16) or 3 (BF16); each value rounded once, to nearest even.
hipError_t launch_round_values(int64_t nnz, const double *src, void *dst, int to, int grid, hipStream_t s);
// Sets x = 0 when b == 0, then (optionally) recomputes ||b - A x|| into the state.
hipError_t launch_cg_finalize(const CsrDev &A, const SpmvTune &t, const double *b, double *x,
                              SolveState *st, double *partials, int true_residual, hipStream_t s);

hipError_t launch_copy(const void *src, void *dst, size_t bytes, int grid, hipStream_t s);
// dst[i] = src[idx[i]], i < m (idx in range).
hipError_t launch_gather(const double *src, const int32_t *idx, double *dst, int64_t m, int grid, hipStream_t s);

// Allocation-free solves (spk_noalloc.hip).  noalloc_scratch_setup: device
// address of this device's scratch array (kNoallocScratchBytes), looked up
// once per device with the device current; later calls return the kept
// address (and the first lookup's error).  launch_fill_zero: bytes (a
// multiple of 16, 16-byte aligned) set to zero by a kernel.
hipError_t noalloc_scratch_setup(int device, void **addr);
hipError_t launch_fill_zero(void *p, size_t bytes, int grid, hipStream_t s);

// CGS (FP64; spk_krylov.hip).  Iteration j of a chunk = dir(j), spmv_v,
// update(j), spmv_r; a chunk of c iterations ends with check(c).  The initial
// residual is launch_cg_init with the shadow residual rt in place of p.
hipError_t launch_cgs_dir(int64_t n, int grid, int spmv_grid, int j, const double *r, double *u, double *p,
                          const double *q, SolveState *st, double *partials, hipStream_t s);
hipError_t launch_cgs_spmv_v(const CsrDev &A, const SpmvTune &t, const double *p, double *v, const double *rt,
                             SolveState *st, double *partials, hipStream_t s);
hipError_t launch_cgs_update(int64_t n, int grid, int spmv_grid, int j, const double *u, const double *v, double *q,
                             double *uh, SolveState *st, double *partials, hipStream_t s);
hipError_t launch_cgs_spmv_r(const CsrDev &A, const SpmvTune &t, const double *uh, double *r, const double *rt,
                             SolveState *st, double *partials, hipStream_t s);
hipError_t launch_cgs_check(SolveState *st, double *partials, int spmv_grid, int count, hipStream_t s);

// Restarted GMRES(m) (spk_gmres.hip).  V holds m + 1 basis vectors, column t
// at V + t * gm_ld(n) elements (16-byte aligned for the packed passes); w is
// one more vector (16-byte aligned), gpart (kMaxKrylov + 1) * kMaxGrid
// doubles.  A solve is begin, then per cycle: cycle_start (r = b - A x
// into v_0, beta, stop test), for j = 0..m-1 step_spmv(j) and step_rest(j),
// then cycle_end (R y = g, x += V y); the host polls after each cycle.
constexpr int64_t gm_ld(int64_t n) { return (n + 63) / 64 * 64; }
hipError_t launch_gm_begin(SolveState *st, GmresState *gs, void *x, double *hist, int64_t hist_cap,
                           int64_t max_iters, hipStream_t s);
// fp32: FP32 basis, w and x (A's values F32, BF16 or F16), else FP64 (F64 values).
hipError_t launch_gm_cycle_start(const CsrDev &A, const SpmvTune &t, const void *b, const void *x, void *V,
                                 SolveState *st, GmresState *gs, double *partials, double tau, int m, bool fp32,
                                 hipStream_t s);
// The same when x = 0 (no product: r = b); grid workgroups of kBlock.
hipError_t launch_gm_cycle_start_zero(int64_t n, int grid, const void *b, void *V, SolveState *st, GmresState *gs,
                                      double *partials, double tau, int m, bool fp32, hipStream_t s);
hipError_t launch_gm_step_spmv(const CsrDev &A, const SpmvTune &t, const void *V, void *w, int j,
                               const SolveState *st, const GmresState *gs, bool fp32, hipStream_t s);
hipError_t launch_gm_step_rest(int64_t n, int grid, void *V, void *w, int j, int m, SolveState *st, GmresState *gs,
                               double *gpart, bool fp32, hipStream_t s);
hipError_t launch_gm_cycle_end(int64_t n, int grid, int m, const void *V, SolveState *st, GmresState *gs, bool fp32,
                               hipStream_t s);

// Jacobi-preconditioned CG (FP64; spk_krylov.hip).  diag_inv runs once per
// plan (flag: one zeroed unsigned, set when a diagonal entry is zero or not
// finite).  Iteration j = launch_cg_spmv_pq, pcg_update(j), pcg_pupdate(j);
// chunks end with launch_cg_chunk_end.
hipError_t launch_diag_inv(const CsrDev &A, double *dinv, unsigned *flag, hipStream_t s);
// Right preconditioning of CGS / GMRES by M = diag(A): out = A M^{-1}
// values (F64, nnz), and x <- M x (to_u = 1) or x <- M^{-1} x (to_u = 0).
hipError_t launch_scale_cols(const CsrDev &A, const double *dinv, double *out, hipStream_t s);
hipError_t launch_jacobi_vec(int64_t n, double *x, const double *dinv, int to_u, hipStream_t s);
hipError_t launch_pcg_init(const CsrDev &A, const SpmvTune &t, const double *b, double *x, const double *dinv,
                           const unsigned *bad_diag, double *r, double *p, SolveState *st, double *partials,
                           double tau, int64_t max_iters, double *hist, int64_t hist_cap, hipStream_t s);
hipError_t launch_pcg_update(int64_t n, int grid, int spmv_grid, int j, double *r, const double *q,
                             const double *dinv, SolveState *st, double *partials, hipStream_t s);
hipError_t launch_pcg_pupdate(int64_t n, int grid, int j, const double *r, const double *dinv, double *p,
                              SolveState *st, double *partials, hipStream_t s);

// Persistent solves (spk_persist.hip): the whole CG solve in one
// cooperative launch, one grid barrier per fused iteration.  A: the matrix of
// the iterations (FP64 values for an FP64 solve; the FP32/BF16/FP16 inner
// values of a mixed solve); outer: the refinement's matrix of a mixed solve
// (same index arrays, FP64 or FP32-exact values), nullptr for FP64.  The
// grid must be co-resident: grid <= persistent_blocks_per_cu(A, outer) * CUs
// (0: no persistent kernel for these types; then use the host loop).  The
// launcher fills the matrix fields of a.  bar: 3 unsigned, [0] and [2] zero
// at launch; afterwards bar[2] != 0 means a barrier waited longer than
// spin_ticks (wall clock) and the solve was abandoned.  An FP64 solve leaves
// its state in a.st as the host loop does (true residual included); a mixed
// solve writes a.res.
hipError_t launch_persistent(const CsrDev &A, const CsrDev *outer, PersistSolve a, int grid, hipStream_t s);
int persistent_blocks_per_cu(const CsrDev &A, const CsrDev *outer);

// Workgroups of the SpMV kernel resident per CU for this tune/type (occupancy API).
int spmv_blocks_per_cu(const CsrDev &A, const SpmvTune &t);

// HIP device of a context (spk_api.cpp).
int ctx_device(const struct ::spk_ctx_s *ctx);

}  // namespace spk

namespace spk {

// One tick: six launches advancing every live slot by one step of its phase.
hipError_t launch_batch_tick(const BatchDev &B, hipStream_t s);
// FP64 -> FP32 values of a newly admitted request.
hipError_t launch_round_f32(int64_t nnz, const double *src, float *dst, int grid, hipStream_t s);
hipError_t launch_narrow_i32(int64_t count, const int64_t *src, int32_t *dst, int grid, hipStream_t s);
int batch_tile_blocks_per_cu();

}  // namespace spk
