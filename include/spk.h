/*
 * spk — sparse Krylov solves on one MI355X (gfx950), C ABI.
 *
 * The operation: a CSR sparse matrix A applied to a vector (SpMV, y = A x;
 * the operator apply of the paper's Section 4.2, benchmarked as a matrix
 * times a random vector in Section 6.1), and Krylov solves of A x = b: the
 * conjugate gradient solve of Section 6.2 (unpreconditioned, or with the
 * scalar Jacobi preconditioner of the Section 3.5 configuration example) and
 * CGS, the other solver benchmarked in Section 6.2, for nonsymmetric A.
 * Solves stop on an iteration cap or on ||r|| <= reduction_factor * ||b||
 * (the "Iteration" and "ResidualNorm" criteria with baseline rhs_norm of the
 * configuration example in Section 3.5, Listing 2).  The solution overwrites the initial guess and
 * a log reports convergence (Section 3.5, around Listing 1).  Value types
 * half/float/double and index types int32/int64 follow Table 1.
 *
 * Conventions for every entry point:
 *  - All matrix and vector pointers are DEVICE pointers owned by the caller.
 *    A plan borrows the CSR arrays until spk_free; the caller must not free
 *    or modify them meanwhile.  A plan owns only what it derives (workspace,
 *    low-precision value copies, tuning results).
 *  - Work is enqueued on the context's HIP stream.  spk_execute_* return
 *    after the work has finished (the log is then valid) unless stated.
 *  - Functions never abort and never throw; they return a status.  On error
 *    spk_last_error(ctx) gives a message.  Non-convergence is NOT an error:
 *    it is reported in spk_log.stop_reason.
 *  - Handles are not thread-safe: one host thread per context at a time.
 */
#ifndef SPK_H
#define SPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPK_OK = 0,
    SPK_ERR_INVALID_ARG = 1,   /* null pointer, bad size, malformed CSR, dtype mismatch */
    SPK_ERR_UNSUPPORTED = 2,   /* valid request the library does not implement */
    SPK_ERR_OUT_OF_MEMORY = 3, /* device or pinned-host allocation failed */
    SPK_ERR_BUDGET = 4,        /* request exceeds a configured memory budget */
    SPK_ERR_DEVICE = 5,        /* a HIP runtime call failed */
    SPK_ERR_INTERNAL = 6
} spk_status;

/* Value types (Table 1 plus bfloat16 storage). */
typedef enum { SPK_F64 = 0, SPK_F32 = 1, SPK_F16 = 2, SPK_BF16 = 3 } spk_dtype;
/* Index types (Table 1).  row_ptr and col_idx types are independent. */
typedef enum { SPK_I32 = 0, SPK_I64 = 1 } spk_itype;

/* CSR well-formedness verdicts, in the order the checks are applied; the
 * first failing check is reported. */
typedef enum {
    SPK_CSR_OK = 0,
    SPK_CSR_BAD_SIZE = 1,    /* negative n_rows, n_cols or nnz */
    SPK_CSR_BAD_FIRST = 2,   /* row_ptr[0] != 0 */
    SPK_CSR_DECREASING = 3,  /* row_ptr[i+1] < row_ptr[i] for some i */
    SPK_CSR_BAD_LAST = 4,    /* row_ptr[n_rows] != nnz */
    SPK_CSR_BAD_COLUMN = 5   /* some col_idx outside [0, n_cols) */
} spk_csr_verdict;

/* Why a solve stopped (spk_log.stop_reason). */
typedef enum {
    SPK_STOP_RUNNING = 0,
    SPK_STOP_CONVERGED = 1,   /* ||r_k|| <= reduction_factor * ||b||, or b = 0 (then x = 0) */
    SPK_STOP_MAX_ITERS = 2,   /* k == max_iters */
    SPK_STOP_BREAKDOWN = 3,   /* CG: p.Ap <= 0 (A not positive definite along p), or a zero
                                 or non-finite diagonal with the Jacobi preconditioner;
                                 CGS: rt.r == 0 or rt.Ap == 0 */
    SPK_STOP_NON_FINITE = 4   /* a NaN or Inf appeared in a norm or inner product */
} spk_stop_reason;

typedef enum {
    SPK_SOLVER_CG = 0,        /* conjugate gradient: A symmetric positive definite */
    SPK_SOLVER_CGS = 1,       /* conjugate gradient squared: general nonsingular A; FP64;
                                 two SpMVs per iteration */
    SPK_SOLVER_GMRES = 2      /* restarted GMRES(krylov_dim): general nonsingular A;
                                 iterations count Arnoldi steps and the stop test
                                 uses the Givens residual estimate (the true residual at each
                                 restart).  With a mixed precision it is the inner solver
                                 of the refinement (GMRES-IR) */
} spk_solver;
typedef enum {
    SPK_PREC_FP64 = 0,        /* FP64 values, vectors and reductions */
    SPK_PREC_MIXED_FP32 = 1,  /* FP32 inner solve (CG or GMRES: FP32 vectors, FP64 reductions)
                                 + FP64 iterative refinement */
    SPK_PREC_MIXED_BF16 = 2,  /* BF16 matrix values in the inner solve, otherwise as MIXED_FP32 */
    SPK_PREC_MIXED_FP16 = 3   /* IEEE binary16 ("half", Table 1) matrix values in the inner solve,
                                 otherwise as MIXED_FP32 */
} spk_precision;
typedef enum { SPK_BASELINE_RHS_NORM = 0 } spk_baseline;
typedef enum {
    SPK_PRECOND_NONE = 0,
    SPK_PRECOND_JACOBI = 1    /* scalar Jacobi, M = diag(A), FP64: CG applies it as PCG; CGS and
                                 GMRES on the right (the plan keeps the values of A M^{-1}).
                                 The stop test stays on the unpreconditioned residual ||r|| */
} spk_precond;
typedef enum {
    SPK_EXEC_AUTO = 0,        /* the library's choice: the host loop, which measured fastest */
    SPK_EXEC_HOST_LOOP = 1,   /* kernels launched from a host loop, status polled per chunk */
    SPK_EXEC_GRAPH = 2,       /* chunks of iterations replayed from a captured HIP graph */
    SPK_EXEC_PERSISTENT = 3   /* FP64 CG: the whole solve in one cooperative launch with grid
                                 barriers (other solves fall back to SPK_EXEC_GRAPH) */
} spk_exec_mode;

typedef struct spk_ctx_s *spk_ctx;
typedef struct spk_plan_s *spk_plan;

/* A CSR matrix in device memory.  row_ptr has n_rows + 1 entries of
 * ptr_type; col_idx and values have nnz entries of idx_type / val_type.
 * Columns within a row may be unsorted; duplicate entries are summed. */
typedef struct {
    int64_t n_rows, n_cols, nnz;
    int32_t ptr_type, idx_type, val_type, reserved;
    const void *row_ptr;
    const void *col_idx;
    const void *values;
} spk_csr;

/* A COO (coordinate) matrix in device memory, the SpMV benchmark's second
 * format (Section 6.1): nnz (row, column, value) triplets in three arrays.
 * Row indices must be non-decreasing (entries sorted by row; any column order
 * within a row; duplicates summed).  row_idx and col_idx share idx_type. */
typedef struct {
    int64_t n_rows, n_cols, nnz;
    int32_t idx_type, val_type;
    const void *row_idx;
    const void *col_idx;
    const void *values;
} spk_coo;

/* Solver configuration; spk_solver_cfg_default fills the defaults noted. */
typedef struct {
    int32_t solver;            /* SPK_SOLVER_CG (or SPK_SOLVER_CGS, SPK_SOLVER_GMRES) */
    int32_t precision;         /* SPK_PREC_FP64 */
    int32_t baseline;          /* SPK_BASELINE_RHS_NORM */
    int32_t precond;           /* SPK_PRECOND_NONE (or SPK_PRECOND_JACOBI) */
    int64_t max_iters;         /* "Iteration" criterion; 1000 (Listings 1-2) */
    double reduction_factor;   /* "ResidualNorm" criterion; 1e-6 (Listings 1-2) */
    int32_t exec_mode;         /* SPK_EXEC_AUTO */
    int32_t chunk_iters;       /* iterations per status poll / graph replay; 0 = auto */
    int32_t record_history;    /* 1: keep ||r_k|| for k = 0..iterations */
    int32_t true_residual;     /* 1: recompute ||b - A x|| at exit (default 1) */
    double inner_reduction;    /* mixed: inner solve reduction factor (default 1e-4) */
    int64_t max_outer;         /* mixed: refinement step cap (default 50) */
    int64_t krylov_dim;        /* GMRES restart length, 1..32 (default 30, Listings 1-2) */
    int64_t reserved[3];
} spk_solver_cfg;

/* What a solve did (the paper's logger). */
typedef struct {
    int64_t iterations;        /* solver iterations (inner iterations summed for mixed) */
    int64_t outer_iterations;  /* refinement steps (mixed), else 0 */
    double implicit_resnorm;   /* ||r_k|| of the recurrence residual at exit */
    double true_resnorm;       /* ||b - A x|| recomputed in FP64 at exit (NaN if not computed) */
    double rhs_norm;           /* ||b|| */
    int32_t converged;         /* stop_reason == SPK_STOP_CONVERGED */
    int32_t stop_reason;       /* spk_stop_reason */
    double elapsed_ms;         /* device time of the execute call (HIP events) */
} spk_log;

/* Tuning decisions a plan made (for reports and tests). */
typedef struct {
    int32_t spmv_kernel;       /* 0 = LDS-staged row tiles, 1 = lanes-per-row vector kernel */
    int32_t lanes;             /* lanes per row of the vector kernel */
    int32_t grid;              /* SpMV workgroups */
    int32_t xcd_remap;         /* tile order: 0 round-robin, 1 XCD eighths, k >= 2 XCD blocks of k tiles */
    int32_t exec_mode;         /* resolved spk_exec_mode */
    int32_t chunk_iters;       /* resolved chunk size */
    int32_t tuned;             /* 1 = chosen by timing candidates, 0 = heuristic/cached */
    int32_t col_codes;         /* bit 0: the row-tile SpMV reads one byte per entry naming
                                  its column offset from the row in a table of at most 256
                                  offsets derived at plan time, in place of col_idx;
                                  bit 1: it also reads packed row pointers (an int64 per
                                  256-row tile, a uint16 offset per row) in place of row_ptr */
    double spmv_ms;            /* measured time of the chosen SpMV (0 if not tuned) */
    int32_t fused_loop;        /* 1 = CG runs one launch per iteration: the SpMV step also forms
                                  the direction from the previous r, q and p at every gathered
                                  column and updates x, r and p (0 = three launches) */
    int32_t nontemporal;       /* 1 = the row-tile SpMV streams the matrix with non-temporal loads */
} spk_plan_info;

/* Fill cfg with the defaults documented in spk_solver_cfg. */
void spk_solver_cfg_default(spk_solver_cfg *cfg);

/* Create a context on HIP device device_id that enqueues on hip_stream
 * (a hipStream_t; NULL = the device's null stream).  *out receives the
 * handle.  The context plays the part of the paper's executor: the object
 * that names the device every operator and vector lives on and runs on
 * (Section 4.1, the Executor; created first in Listing 1).
 * Errors: INVALID_ARG (out NULL, bad device), DEVICE. */
spk_status spk_init(int device_id, void *hip_stream, spk_ctx *out);

/* Destroy a context.  All its plans must have been freed.  NULL is a no-op. */
spk_status spk_finalize(spk_ctx ctx);

/* Message for the last error on this context (never NULL). */
const char *spk_last_error(spk_ctx ctx);

/* Static name of a status code. */
const char *spk_status_string(spk_status s);

/* Validate a device CSR matrix (row_ptr, col_idx) on the GPU.  *verdict
 * receives an spk_csr_verdict.  Returns OK whatever the verdict; INVALID_ARG
 * only for null handle/pointers or unknown index types. */
spk_status spk_csr_check(spk_ctx ctx, const spk_csr *A, int32_t *verdict);

/* nnz-balanced row partition into parts pieces, computed on the GPU:
 *   split[j] = min { i : row_ptr[i] >= floor(j * nnz / parts) } (j < parts),
 *   split[parts] = n_rows.
 * split_dev is a device array of parts + 1 int64.  A must be valid. */
spk_status spk_partition(spk_ctx ctx, const spk_csr *A, int64_t parts, int64_t *split_dev);

/* Plan y = A x.  Validates A (INVALID_ARG if malformed) and picks the SpMV
 * kernel.  x and y have val_type F64 -> FP64, else FP32 (F16/BF16 values are
 * widened to FP32; accumulation is in the vector type). */
spk_status spk_plan_spmv(spk_ctx ctx, const spk_csr *A, spk_plan *out);

/* Validate a device COO matrix on the GPU.  *verdict receives an
 * spk_csr_verdict: BAD_SIZE for a negative size, BAD_FIRST for a row index
 * out of range, BAD_COLUMN for a column index out of range (checked in that
 * order); *row_sorted = 1 when the row indices are non-decreasing.  Returns
 * OK whatever the verdict; INVALID_ARG for null pointers or unknown types. */
spk_status spk_coo_check(spk_ctx ctx, const spk_coo *A, int32_t *verdict, int32_t *row_sorted);

/* Plan y = A x for a COO matrix (executed with spk_execute_spmv).  Validates
 * A (INVALID_ARG if malformed or not sorted by row), then derives on the GPU
 * the row pointer of the same matrix (n_rows + 1 entries, int32 when
 * nnz < 2^31, else int64; owned by the plan) so that each product runs the
 * CSR kernels over the caller's col_idx and values, which the plan borrows.
 * Results equal those of spk_plan_spmv on the corresponding CSR matrix. */
spk_status spk_plan_spmv_coo(spk_ctx ctx, const spk_coo *A, spk_plan *out);

/* Plan a solve of A x = b: the counterpart of generating a solver operator
 * for a system matrix from a configured factory (the generic solver entry
 * point of Section 5, instantiated through a LinOp factory as in Section
 * 4.2; the factory and its stopping criteria in Listings 1-2).  A must be
 * square and valid.
 * FP64 precision
 * needs val_type F64; the mixed precisions accept F64 values (the plan keeps
 * an FP32, BF16 or FP16 copy for the inner solve, each value rounded once to
 * nearest even) or, for MIXED_FP32, F32 values (taken as exact).
 * CGS and the Jacobi preconditioner are FP64 only; GMRES runs in the host
 * loop, in FP64 or as the inner solver of a mixed precision (its basis then
 * holds (krylov_dim + 1) n floats); a Jacobi plan computes 1 / diag(A) (and for CGS and GMRES a
 * scaled copy of the values, nnz doubles); a zero or non-finite diagonal
 * entry makes every solve of the plan stop with SPK_STOP_BREAKDOWN, x
 * unchanged.
 * Errors: INVALID_ARG, UNSUPPORTED (other solver / precision /
 * preconditioner combinations), OUT_OF_MEMORY. */
spk_status spk_plan_solve(spk_ctx ctx, const spk_csr *A, const spk_solver_cfg *cfg, spk_plan *out);

/* y = A x with the plan's matrix (a matrix operator's apply is the SpMV,
 * Section 4.2; benchmarked in Section 6.1); x has n_cols entries, y has
 * n_rows. */
spk_status spk_execute_spmv(spk_plan plan, const void *x, void *y);

/* Solve A x = b: the solver's apply(b, x), which overwrites the initial
 * guess x with the solution and returns the logger's record (Section 3.5,
 * Listing 1).  b (n entries, FP64) is read; x (n entries, FP64) holds the
 * initial guess on entry and the last iterate on exit.  log may be NULL. */
spk_status spk_execute_solve(spk_plan plan, const void *b, void *x, spk_log *log);

/* Copy the residual-norm history of the last solve (needs record_history):
 * up to cap values into host array out; *count receives iterations + 1. */
spk_status spk_plan_history(spk_plan plan, double *out, int64_t cap, int64_t *count);

/* Report the plan's tuning decisions. */
spk_status spk_plan_get_info(spk_plan plan, spk_plan_info *info);

/* Per-kernel timing: with on = k >= 1, every k-th launch of the plan's
 * dominant SpMV kernel (launches 0, k, 2k, ... of each solve, counting
 * only launches that did work) is bracketed by HIP events on the context
 * stream; on <= 0 turns timing off.  Stats return the summed device time
 * (ms) and the count of timed launches since the last reset. */
spk_status spk_plan_set_profiling(spk_plan plan, int32_t on);
spk_status spk_plan_kernel_stats(spk_plan plan, double *total_ms, int64_t *launches);

/* Release a plan and everything it derived.  NULL is a no-op. */
spk_status spk_free(spk_plan plan);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one FP64
 * CG solve of A x = b (plan + execute + free in one call) whose workspace is
 * a fixed scratch array the library holds on each GPU until the process
 * ends, so the call makes no hipMalloc, hipFree or other allocating call.
 * cfg (NULL = defaults) must ask for CG, FP64, no preconditioner, AUTO or
 * HOST_LOOP execution and no history.  A: square, F64 values, at most
 * spk_noalloc_max_rows() rows (the scratch holds the solve state, the
 * reduction partials and the vectors of n doubles: r, p, q, and their second
 * buffers when the solve runs one launch per iteration, as systems of up to
 * 2^20 rows do); the caller's arrays
 * are borrowed for the call only.  b and x as for spk_execute_solve.  The
 * launch shape is one an earlier plan of the same shape tuned on this
 * context (never tuned here), else the heuristic one, so a solve after such
 * a plan runs the same kernels and gives the same result (for matrices of
 * fewer than 2^22 entries: larger plans also derive column codes, which this
 * solve does not, so its launch shape and rounding can differ there).  Every call on one
 * GPU shares that GPU's scratch, which keeps the last call's contents (the
 * call clears what must start at zero): calls that overlap on one GPU, from
 * any context or stream, race and must not be issued.  Synchronises the
 * context stream before returning.
 * Errors: INVALID_ARG (malformed or non-square A, too many rows, null
 * vectors), UNSUPPORTED (other configurations), DEVICE. */
spk_status spk_solve_noalloc(spk_ctx ctx, const spk_csr *A, const spk_solver_cfg *cfg, const void *b, void *x,
                             spk_log *log);

/* Largest n_rows spk_solve_noalloc accepts (its scratch is 64 MiB per GPU). */
int64_t spk_noalloc_max_rows(void);

/* Plain device-to-device copy of bytes (multiple of 16, 16-byte aligned
 * pointers) with the library's streaming copy kernel; *ms receives its
 * device time.  Used to measure the achievable HBM bandwidth. */
spk_status spk_stream_copy(spk_ctx ctx, const void *src, void *dst, size_t bytes, double *ms);

/* Random-gather calibration: dst[i] = src[idx[i]] for i < m (device arrays:
 * n_src doubles, m int32 indices in [0, n_src), m doubles) with the
 * library's gather kernel, indices and results streamed, the source read at
 * the given positions; *ms receives its device time.  With uniform random
 * indices it measures the rate of the scattered 8-byte reads an SpMV of an
 * irregular pattern makes of its input vector (a ceiling beside the HBM
 * bandwidth spk_stream_copy measures).  The indices are range-checked on the
 * GPU first.  Errors: INVALID_ARG (null pointers, sizes, an index out of
 * range), OUT_OF_MEMORY, DEVICE. */
spk_status spk_gather_probe(spk_ctx ctx, const double *src, int64_t n_src, const int32_t *idx, int64_t m,
                            double *dst, double *ms);

/* ---------------------------------------------------------------- serving
 * A continuous-batching solve server.  Requests of uneven sizes arrive from
 * any host thread; a worker thread admits each into a free slot once its
 * workspace fits the HBM budget, and every live request advances in the same
 * batched launches, on per-request 256-row tiles: a SPK_PREC_MIXED_FP32
 * request by FP32 CG with FP64 dot products and FP64 iterative refinement
 * (the mixed-precision solve above), a SPK_PREC_FP64 request by FP64 CG
 * (Algorithm 1) to ||r|| <= reduction_factor ||b|| on the recurrence
 * residual, then confirmed on the true residual b - A x (a restart from it
 * if the test fails there).  Requests that arrive while others run join between tick
 * batches.  A request's result is bitwise independent of which other
 * requests share the batch.  Small systems being overhead-bound is the
 * paper's observation (Sections 6.1-6.2); batching many of them into one
 * launch per step is how the library serves them. */
typedef struct spk_server_s *spk_server;

typedef struct {
    int64_t submitted, admitted, completed, failed;
    int64_t ticks;          /* batched steps run */
    int64_t peak_slots;     /* most requests live at once */
    int64_t peak_bytes;     /* most workspace bytes held at once */
    int64_t budget_bytes;
    int64_t max_slots;
    int64_t peak_device_bytes; /* most device bytes the request pool held at once (blocks in use
                                  plus cached ones); never above budget_bytes */
} spk_server_stats;

/* Workspace bytes one SPK_PREC_MIXED_FP32 request of n unknowns and nnz
 * stored entries needs (counted against the budget).  Pure host computation. */
size_t spk_server_request_bytes(int64_t n, int64_t nnz);

/* As spk_server_request_bytes for a request of the given precision
 * (SPK_PREC_MIXED_FP32, or SPK_PREC_FP64: four FP64 vectors and no value
 * copy) on 32-bit indices; 0 for a precision the server does not run. */
size_t spk_server_request_bytes_prec(int32_t precision, int64_t n, int64_t nnz);

/* Workspace bytes of a request of matrix A (its sizes and index types; the
 * pointers are not read) at the given precision: as
 * spk_server_request_bytes_prec, plus 32-bit copies of 64-bit row pointers
 * (n + 1) and columns (nnz), each rounded up to 256 bytes.  0 for index
 * types or a precision the server does not take. */
size_t spk_server_request_bytes_csr(const spk_csr *A, int32_t precision);

/* Create a server on the context's device with an HBM budget for request
 * workspace and at most max_slots live requests.  cfg (the default of every
 * request): solver CG, no preconditioner, precision SPK_PREC_MIXED_FP32 or
 * SPK_PREC_FP64; reduction_factor is the FP64 stop test
 * ||b - A x|| <= reduction_factor ||b||, inner_reduction the mixed inner
 * CG's, max_iters caps inner iterations per request, max_outer refinement
 * steps (restarts of an FP64 request).
 * Errors: INVALID_ARG, UNSUPPORTED, OUT_OF_MEMORY. */
spk_status spk_server_create(spk_ctx ctx, size_t hbm_budget_bytes, int32_t max_slots, const spk_solver_cfg *cfg,
                             spk_server *out);

/* Queue a solve of A x = b (device pointers; A square with int32 or int64
 * row_ptr and col_idx and F64 values; x holds the initial guess and
 * receives the solution).  64-bit indices are narrowed into the request's
 * workspace at admission, so n and nnz must stay below 2^31 - 1.  The caller
 * keeps A, b, x alive and untouched until the request is done.  *ticket
 * identifies it.  Errors: INVALID_ARG, UNSUPPORTED (index or value types,
 * 64-bit indices past 2^31 - 1), BUDGET (the request alone exceeds the
 * budget).  A malformed CSR is detected on the GPU before admission and
 * reported by poll. */
spk_status spk_server_submit(spk_server srv, const spk_csr *A, const void *b, void *x, uint64_t *ticket);

/* As spk_server_submit, with this request's own solver configuration (its
 * reduction_factor, inner_reduction, max_iters, max_outer and precision
 * (MIXED_FP32 or FP64); solver CG and no preconditioner), so one
 * server mixes requests with different tolerances and precisions (the
 * per-solve stopping criteria of Listing 2).  cfg NULL = the server's configuration.
 * Errors: as spk_server_submit, plus INVALID_ARG / UNSUPPORTED for cfg. */
spk_status spk_server_submit_cfg(spk_server srv, const spk_csr *A, const void *b, void *x, const spk_solver_cfg *cfg,
                                 uint64_t *ticket);

/* Non-blocking: *done = 1 once the request finished; then log and
 * *latency_ns (submission to completion, host steady clock) are filled and
 * the return value is the request's status (OK, INVALID_ARG for a malformed
 * matrix, BUDGET, DEVICE). */
spk_status spk_server_poll(spk_server srv, uint64_t ticket, int32_t *done, spk_log *log, int64_t *latency_ns);

/* Block until every submitted request is done. */
spk_status spk_server_drain(spk_server srv);

spk_status spk_server_get_stats(spk_server srv, spk_server_stats *stats);
const char *spk_server_last_error(spk_server srv);

/* Finish all queued and live requests, then release the server. */
spk_status spk_server_destroy(spk_server srv);

#ifdef __cplusplus
}
#endif

#endif /* SPK_H */
