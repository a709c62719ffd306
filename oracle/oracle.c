/*
 * FP64 CPU oracle for the sparse Krylov solve.  TEST INFRASTRUCTURE ONLY:
 * nothing in the product path may link, load or call this file.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Plain, slow, single-threaded, obviously correct.  Compiled with
 * -O2 -ffp-contract=off and no fast-math, so every expression rounds exactly
 * as written.  Shares no code with the HIP path.
 *
 * What the paper fixes and what it leaves open:
 *  - A matrix operator's apply is a sparse matrix-vector product (Section 4.2)
 *    and the SpMV benchmark multiplies a sparse matrix by a random vector
 *    (Section 6.1).  The oracle's SpMV is the textbook CSR definition,
 *    summed in storage order.
 *  - The solver benchmark is conjugate gradient on A x = b with b all ones,
 *    x0 zero and no preconditioner (Section 6.2); the paper names CG but does
 *    not print it, so the oracle takes the Hestenes-Stiefel iteration as in
 *    Saad, "Iterative Methods for Sparse Linear Systems", 2nd ed., Alg. 6.18.
 *  - Stopping: an iteration cap OR a residual-norm reduction relative to the
 *    right-hand-side norm (the criteria list of the configuration example in
 *    Section 3.5, Listing 2: "Iteration" max_iters and "ResidualNorm" with
 *    reduction_factor and baseline rhs_norm).  Readings taken where the paper
 *    is silent: the recurrence residual is tested, in the Euclidean norm, with
 *    an inclusive comparison; the test runs once before the first iteration
 *    and after every update; ||b|| = 0 returns x = 0 as converged; p.q <= 0 is
 *    a breakdown; a non-finite scalar stops with a non-finite verdict.
 *  - CGS is among the solvers the paper benchmarks against its baselines
 *    (Section 6.2) without printing the iteration; the oracle takes the
 *    unpreconditioned template of Barrett et al. (1994) with shadow residual
 *    r0 and the same stop tests; an exact zero rho or sigma is a breakdown.
 *  - The SpMV benchmark also runs on the coordinate (COO) format (Section
 *    6.1); the oracle's COO product is its definition, accumulated in
 *    storage order.
 *  - GMRES is the solver of the paper's usage examples (Listings 1-2, with a
 *    Krylov dimension) and of its solver benchmarks (Section 6.2); the
 *    oracle takes textbook restarted GMRES(m) with modified Gram-Schmidt and
 *    Givens rotations, tests the rotation residual estimate after every
 *    Arnoldi step and the true residual at each restart.
 *  - The scalar Jacobi preconditioner appears in the configuration example
 *    (Section 3.5, Listing 2, block size 1); the oracle applies it as
 *    z = r / diag(A) inside textbook PCG (Saad, Alg. 9.1) and keeps the stop
 *    test on the unpreconditioned residual norm.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Stop reasons (numbering mirrored, independently, by the library). */
enum { ORC_RUNNING = 0, ORC_CONVERGED = 1, ORC_MAX_ITERS = 2, ORC_BREAKDOWN = 3, ORC_NON_FINITE = 4 };

/* CSR validation verdicts, in the order the checks are applied. */
enum { ORC_CSR_OK = 0, ORC_CSR_BAD_SIZE = 1, ORC_CSR_BAD_FIRST = 2, ORC_CSR_DECREASING = 3,
       ORC_CSR_BAD_LAST = 4, ORC_CSR_BAD_COLUMN = 5 };

typedef struct {
    int64_t iterations;
    int32_t stop_reason;
    int32_t reserved;
    double rhs_norm;          /* ||b||_2 */
    double implicit_resnorm;  /* ||r_k||_2 of the recurrence residual at exit */
    double true_resnorm;      /* ||b - A x||_2 recomputed at exit */
} orc_cg_result;

/* A CSR matrix is well formed when: sizes are non-negative, row_ptr[0] = 0,
 * row_ptr is non-decreasing, row_ptr[n] = nnz and every column is in [0, n_cols). */
int orc_csr_validate(int64_t n_rows, int64_t n_cols, int64_t nnz,
                     const int64_t *row_ptr, const int64_t *col) {
    if (n_rows < 0 || n_cols < 0 || nnz < 0) return ORC_CSR_BAD_SIZE;
    if (row_ptr[0] != 0) return ORC_CSR_BAD_FIRST;
    for (int64_t i = 0; i < n_rows; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return ORC_CSR_DECREASING;
    if (row_ptr[n_rows] != nnz) return ORC_CSR_BAD_LAST;
    for (int64_t k = 0; k < nnz; ++k)
        if (col[k] < 0 || col[k] >= n_cols) return ORC_CSR_BAD_COLUMN;
    return ORC_CSR_OK;
}

/* y_i = sum over the stored entries k of row i of val[k] * x[col[k]]. */
void orc_spmv(int64_t n_rows, const int64_t *row_ptr, const int64_t *col,
              const double *val, const double *x, double *y) {
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += val[k] * x[col[k]];
        y[i] = s;
    }
}

/* COO SpMV: y = 0, then y[row[k]] += val[k] * x[col[k]] for k = 0..nnz-1 in
 * storage order (any entry order; duplicates summed). */
void orc_coo_spmv(int64_t n_rows, int64_t nnz, const int64_t *row, const int64_t *col,
                  const double *val, const double *x, double *y) {
    for (int64_t i = 0; i < n_rows; ++i) y[i] = 0.0;
    for (int64_t k = 0; k < nnz; ++k) y[row[k]] += val[k] * x[col[k]];
}

/* A COO matrix is well formed when sizes are non-negative and every row and
 * column index is in range.  Checks in this order, each over all entries:
 * sizes (BAD_SIZE), row indices (BAD_FIRST), column indices (BAD_COLUMN).
 * row_sorted reports whether the row indices are non-decreasing. */
int orc_coo_validate(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row, const int64_t *col,
                     int *row_sorted) {
    *row_sorted = 1;
    if (n_rows < 0 || n_cols < 0 || nnz < 0) return ORC_CSR_BAD_SIZE;
    for (int64_t k = 1; k < nnz; ++k)
        if (row[k] < row[k - 1]) *row_sorted = 0;
    for (int64_t k = 0; k < nnz; ++k)
        if (row[k] < 0 || row[k] >= n_rows) return ORC_CSR_BAD_FIRST;
    for (int64_t k = 0; k < nnz; ++k)
        if (col[k] < 0 || col[k] >= n_cols) return ORC_CSR_BAD_COLUMN;
    return ORC_CSR_OK;
}

/* (|A| |x|)_i, the scale of the componentwise rounding-error bound of SpMV. */
void orc_spmv_abs(int64_t n_rows, const int64_t *row_ptr, const int64_t *col,
                  const double *val, const double *x, double *y) {
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += fabs(val[k]) * fabs(x[col[k]]);
        y[i] = s;
    }
}

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* r = b - A x */
void orc_residual(int64_t n, const int64_t *row_ptr, const int64_t *col, const double *val,
                  const double *b, const double *x, double *r) {
    orc_spmv(n, row_ptr, col, val, x, r);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
}

/* Sum over the rows of a block of (b_i - sum_k val[k] x[col[k]])^2: the
 * squared 2-norm of the residual b - A x that the ResidualNorm criterion
 * measures (Section 3.5, Listing 2), restricted to the block's rows.  The
 * block's column indices address the whole x, so a matrix too large to hold
 * can be visited block by block; rows in order, each row's products summed
 * in storage order, squares accumulated in row order. */
double orc_residual_sumsq(int64_t n_rows, const int64_t *row_ptr, const int64_t *col, const double *val,
                          const double *b, const double *x) {
    double acc = 0.0;
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += val[k] * x[col[k]];
        const double r = b[i] - s;
        acc += r * r;
    }
    return acc;
}

/*
 * Conjugate gradient (Hestenes-Stiefel).  x holds the initial guess on entry
 * and the last iterate on exit.  hist (optional, max_iters+1 entries) receives
 * ||r_k||_2 for k = 0..iterations.  Returns the stop reason.
 *
 *   r0 = b - A x0, p0 = r0, rho0 = r0.r0
 *   for k = 0, 1, ...:
 *     q = A p_k;  alpha = rho_k / (p_k.q)
 *     x_{k+1} = x_k + alpha p_k;  r_{k+1} = r_k - alpha q
 *     rho_{k+1} = r_{k+1}.r_{k+1}
 *     beta = rho_{k+1} / rho_k;  p_{k+1} = r_{k+1} + beta p_k
 * with the stop test on sqrt(rho) <= tau ||b|| or k == max_iters.
 */
int orc_cg(int64_t n, const int64_t *row_ptr, const int64_t *col, const double *val,
           const double *b, double *x, double tau, int64_t max_iters,
           orc_cg_result *res, double *hist) {
    double *r = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *q = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int64_t k = 0;
    int reason = ORC_RUNNING;
    double rho = 0.0, resnorm = 0.0;
    const double bnorm = sqrt(dot(n, b, b));
    res->rhs_norm = bnorm;

    if (!isfinite(bnorm)) {
        reason = ORC_NON_FINITE;
        resnorm = bnorm;
        goto done;
    }
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        reason = ORC_CONVERGED;
        resnorm = 0.0;
        if (hist) hist[0] = 0.0;
        goto done;
    }
    orc_residual(n, row_ptr, col, val, b, x, r);
    for (int64_t i = 0; i < n; ++i) p[i] = r[i];
    rho = dot(n, r, r);
    resnorm = sqrt(rho);
    if (hist) hist[0] = resnorm;
    if (!isfinite(rho)) reason = ORC_NON_FINITE;
    else if (resnorm <= tau * bnorm) reason = ORC_CONVERGED;
    else if (k >= max_iters) reason = ORC_MAX_ITERS;

    while (reason == ORC_RUNNING) {
        orc_spmv(n, row_ptr, col, val, p, q);
        const double pq = dot(n, p, q);
        if (!isfinite(pq)) { reason = ORC_NON_FINITE; break; }
        if (pq <= 0.0) { reason = ORC_BREAKDOWN; break; }
        const double alpha = rho / pq;
        for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
        for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
        const double rho_new = dot(n, r, r);
        k += 1;
        resnorm = sqrt(rho_new);
        if (hist) hist[k] = resnorm;
        if (!isfinite(rho_new)) { reason = ORC_NON_FINITE; break; }
        if (resnorm <= tau * bnorm) { reason = ORC_CONVERGED; break; }
        if (k >= max_iters) { reason = ORC_MAX_ITERS; break; }
        const double beta = rho_new / rho;
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }

done:
    res->iterations = k;
    res->stop_reason = reason;
    res->implicit_resnorm = resnorm;
    if (reason != ORC_NON_FINITE && n > 0) {
        orc_residual(n, row_ptr, col, val, b, x, r);
        res->true_resnorm = sqrt(dot(n, r, r));
    } else {
        res->true_resnorm = (n > 0) ? NAN : 0.0;
    }
    free(r); free(p); free(q);
    return reason;
}

/*
 * Conjugate gradient squared (Sonneveld 1989), unpreconditioned, in the form
 * of Barrett et al., "Templates for the Solution of Linear Systems" (1994),
 * with the shadow residual rt = r0.  Same argument conventions, stop tests
 * and stop reasons as orc_cg; one iteration = two products with A.
 *
 *   r0 = b - A x0, rt = r0
 *   for i = 1, 2, ...:
 *     rho_{i-1} = rt.r_{i-1}                 (zero: breakdown)
 *     i = 1: u = r_0, p = u
 *     else:  beta = rho_{i-1} / rho_{i-2}
 *            u = r_{i-1} + beta q,  p = u + beta (q + beta p)
 *     v = A p;  sigma = rt.v                  (zero: breakdown)
 *     alpha = rho_{i-1} / sigma
 *     q = u - alpha v;  uh = u + q
 *     x_i = x_{i-1} + alpha uh;  r_i = r_{i-1} - alpha A uh
 * with the stop test on ||r_i|| <= tau ||b|| or i == max_iters.
 */
static int cgs_core(int64_t n, const int64_t *row_ptr, const int64_t *col, const double *val,
                    const double *b, double *x, double tau, int64_t max_iters,
                    orc_cg_result *res, double *hist, const double *d) {
    const size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r = (double *)malloc(bytes), *rt = (double *)malloc(bytes), *p = (double *)malloc(bytes);
    double *u = (double *)malloc(bytes), *q = (double *)malloc(bytes), *v = (double *)malloc(bytes);
    double *uh = (double *)malloc(bytes), *qh = (double *)malloc(bytes);
    int64_t k = 0;
    int reason = ORC_RUNNING;
    double rho_prev = 0.0, resnorm = 0.0;
    const double bnorm = sqrt(dot(n, b, b));
    res->rhs_norm = bnorm;

    if (!isfinite(bnorm)) {
        reason = ORC_NON_FINITE;
        resnorm = bnorm;
        goto done;
    }
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        reason = ORC_CONVERGED;
        resnorm = 0.0;
        if (hist) hist[0] = 0.0;
        goto done;
    }
    orc_residual(n, row_ptr, col, val, b, x, r);
    for (int64_t i = 0; i < n; ++i) rt[i] = r[i];
    resnorm = sqrt(dot(n, r, r));
    if (hist) hist[0] = resnorm;
    if (!isfinite(resnorm)) reason = ORC_NON_FINITE;
    else if (resnorm <= tau * bnorm) reason = ORC_CONVERGED;
    else if (k >= max_iters) reason = ORC_MAX_ITERS;

    while (reason == ORC_RUNNING) {
        const double rho = dot(n, rt, r);
        if (!isfinite(rho)) { reason = ORC_NON_FINITE; break; }
        if (rho == 0.0) { reason = ORC_BREAKDOWN; break; }
        if (k == 0) {
            for (int64_t i = 0; i < n; ++i) u[i] = r[i];
            for (int64_t i = 0; i < n; ++i) p[i] = u[i];
        } else {
            const double beta = rho / rho_prev;
            for (int64_t i = 0; i < n; ++i) u[i] = r[i] + beta * q[i];
            for (int64_t i = 0; i < n; ++i) p[i] = u[i] + beta * (q[i] + beta * p[i]);
        }
        if (d) {   /* v = A M^{-1} p */
            for (int64_t i = 0; i < n; ++i) qh[i] = p[i] / d[i];
            orc_spmv(n, row_ptr, col, val, qh, v);
        } else {
            orc_spmv(n, row_ptr, col, val, p, v);
        }
        const double sigma = dot(n, rt, v);
        if (!isfinite(sigma)) { reason = ORC_NON_FINITE; break; }
        if (sigma == 0.0) { reason = ORC_BREAKDOWN; break; }
        const double alpha = rho / sigma;
        for (int64_t i = 0; i < n; ++i) q[i] = u[i] - alpha * v[i];
        for (int64_t i = 0; i < n; ++i) uh[i] = u[i] + q[i];
        if (d)     /* uh = M^{-1} (u + q) */
            for (int64_t i = 0; i < n; ++i) uh[i] = uh[i] / d[i];
        for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * uh[i];
        orc_spmv(n, row_ptr, col, val, uh, qh);
        for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * qh[i];
        k += 1;
        resnorm = sqrt(dot(n, r, r));
        if (hist) hist[k] = resnorm;
        if (!isfinite(resnorm)) { reason = ORC_NON_FINITE; break; }
        if (resnorm <= tau * bnorm) { reason = ORC_CONVERGED; break; }
        if (k >= max_iters) { reason = ORC_MAX_ITERS; break; }
        rho_prev = rho;
    }

done:
    res->iterations = k;
    res->stop_reason = reason;
    res->implicit_resnorm = resnorm;
    if (reason != ORC_NON_FINITE && n > 0) {
        orc_residual(n, row_ptr, col, val, b, x, r);
        res->true_resnorm = sqrt(dot(n, r, r));
    } else {
        res->true_resnorm = (n > 0) ? NAN : 0.0;
    }
    free(r); free(rt); free(p); free(u); free(q); free(v); free(uh); free(qh);
    return reason;
}

int orc_cgs(int64_t n, const int64_t *row_ptr, const int64_t *col, const double *val,
            const double *b, double *x, double tau, int64_t max_iters,
            orc_cg_result *res, double *hist) {
    return cgs_core(n, row_ptr, col, val, b, x, tau, max_iters, res, hist, NULL);
}


/*
 * Diagonal of A: d_i = sum of the stored entries of row i in column i (0 when
 * there is none).
 */
void orc_diagonal(int64_t n, const int64_t *row_ptr, const int64_t *col, const double *val, double *d) {
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col[k] == i) s += val[k];
        d[i] = s;
    }
}

/*
 * CGS (here) and GMRES(m) (after gmres_core) with the scalar Jacobi
 * preconditioner M = diag(A) applied on the right (Barrett et al.'s preconditioned CGS template; Saad, Alg. 9.5
 * for GMRES): the iteration runs on A M^{-1} and the residual it tests is
 * the unpreconditioned b - A x.  A zero or non-finite diagonal entry stops
 * with ORC_BREAKDOWN before the first iteration, x unchanged (after the
 * non-finite-||b|| check, as in orc_pcg_jacobi).
 */
static int jacobi_diag_ok(int64_t n, const int64_t *row_ptr, const int64_t *col, const double *val,
                          const double *b, double *x, orc_cg_result *res, double **d_out) {
    const double bnorm = sqrt(dot(n, b, b));
    double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    orc_diagonal(n, row_ptr, col, val, d);
    int ok = isfinite(bnorm) ? 1 : 0;   /* a non-finite ||b|| is left to the solver's own check */
    for (int64_t i = 0; ok && i < n; ++i)
        if (d[i] == 0.0 || !isfinite(d[i])) ok = -1;
    if (ok == -1) {
        res->iterations = 0;
        res->stop_reason = ORC_BREAKDOWN;
        res->rhs_norm = bnorm;
        res->implicit_resnorm = NAN;
        double *r = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        orc_residual(n, row_ptr, col, val, b, x, r);
        res->true_resnorm = sqrt(dot(n, r, r));
        free(r);
        free(d);
        *d_out = NULL;
        return 0;
    }
    *d_out = d;
    return 1;
}

int orc_cgs_jacobi(int64_t n, const int64_t *row_ptr, const int64_t *col, const double *val,
                   const double *b, double *x, double tau, int64_t max_iters,
                   orc_cg_result *res, double *hist) {
    double *d = NULL;
    if (!jacobi_diag_ok(n, row_ptr, col, val, b, x, res, &d)) return res->stop_reason;
    const int reason = cgs_core(n, row_ptr, col, val, b, x, tau, max_iters, res, hist, d);
    free(d);
    return reason;
}

/*
 * Conjugate gradient with the scalar Jacobi preconditioner M = diag(A)
 * (Saad, Alg. 9.1, with z = M^{-1} r computed as r_i / d_i).  Same
 * conventions as orc_cg; the stop test uses the unpreconditioned recurrence
 * residual ||r_k||.  A zero or non-finite diagonal entry returns
 * ORC_BREAKDOWN before the first iteration with x unchanged.
 *
 *   r0 = b - A x0, z0 = M^{-1} r0, p0 = z0, rho0 = r0.z0
 *   for k = 0, 1, ...:
 *     q = A p_k;  alpha = rho_k / (p_k.q)             (p.q <= 0: breakdown)
 *     x_{k+1} = x_k + alpha p_k;  r_{k+1} = r_k - alpha q
 *     z_{k+1} = M^{-1} r_{k+1};  rho_{k+1} = r_{k+1}.z_{k+1}
 *     beta = rho_{k+1} / rho_k;  p_{k+1} = z_{k+1} + beta p_k
 */
int orc_pcg_jacobi(int64_t n, const int64_t *row_ptr, const int64_t *col, const double *val,
                   const double *b, double *x, double tau, int64_t max_iters,
                   orc_cg_result *res, double *hist) {
    const size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r = (double *)malloc(bytes), *z = (double *)malloc(bytes), *p = (double *)malloc(bytes);
    double *q = (double *)malloc(bytes), *d = (double *)malloc(bytes);
    int64_t k = 0;
    int reason = ORC_RUNNING;
    double rho = 0.0, resnorm = 0.0;
    const double bnorm = sqrt(dot(n, b, b));
    res->rhs_norm = bnorm;

    if (!isfinite(bnorm)) {
        reason = ORC_NON_FINITE;
        resnorm = bnorm;
        goto done;
    }
    orc_diagonal(n, row_ptr, col, val, d);
    for (int64_t i = 0; i < n; ++i) {
        if (d[i] == 0.0 || !isfinite(d[i])) {
            reason = ORC_BREAKDOWN;
            resnorm = NAN;
            goto done;
        }
    }
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        reason = ORC_CONVERGED;
        resnorm = 0.0;
        if (hist) hist[0] = 0.0;
        goto done;
    }
    orc_residual(n, row_ptr, col, val, b, x, r);
    for (int64_t i = 0; i < n; ++i) z[i] = r[i] / d[i];
    for (int64_t i = 0; i < n; ++i) p[i] = z[i];
    rho = dot(n, r, z);
    resnorm = sqrt(dot(n, r, r));
    if (hist) hist[0] = resnorm;
    if (!isfinite(rho) || !isfinite(resnorm)) reason = ORC_NON_FINITE;
    else if (resnorm <= tau * bnorm) reason = ORC_CONVERGED;
    else if (k >= max_iters) reason = ORC_MAX_ITERS;

    while (reason == ORC_RUNNING) {
        orc_spmv(n, row_ptr, col, val, p, q);
        const double pq = dot(n, p, q);
        if (!isfinite(pq)) { reason = ORC_NON_FINITE; break; }
        if (pq <= 0.0) { reason = ORC_BREAKDOWN; break; }
        const double alpha = rho / pq;
        for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
        for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
        for (int64_t i = 0; i < n; ++i) z[i] = r[i] / d[i];
        const double rho_new = dot(n, r, z);
        k += 1;
        resnorm = sqrt(dot(n, r, r));
        if (hist) hist[k] = resnorm;
        if (!isfinite(rho_new) || !isfinite(resnorm)) { reason = ORC_NON_FINITE; break; }
        if (resnorm <= tau * bnorm) { reason = ORC_CONVERGED; break; }
        if (k >= max_iters) { reason = ORC_MAX_ITERS; break; }
        const double beta = rho_new / rho;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }

done:
    res->iterations = k;
    res->stop_reason = reason;
    res->implicit_resnorm = resnorm;
    if (reason != ORC_NON_FINITE && n > 0) {
        orc_residual(n, row_ptr, col, val, b, x, r);
        res->true_resnorm = sqrt(dot(n, r, r));
    } else {
        res->true_resnorm = (n > 0) ? NAN : 0.0;
    }
    free(r); free(z); free(p); free(q); free(d);
    return reason;
}

/*
 * Restarted GMRES(m), unpreconditioned (Saad, Alg. 6.9 with the Givens
 * rotations of Sec. 6.5.3; Arnoldi by modified Gram-Schmidt).  Same argument
 * conventions and stop reasons as orc_cg; `iterations` counts Arnoldi steps
 * over all cycles and hist[k] holds the residual-norm estimate |g_{k}|
 * after step k (hist[0] = ||r_0||).  Each cycle:
 *
 *   r = b - A x, beta = ||r||  (stop here if beta <= tau ||b||)
 *   v_0 = r / beta, g = beta e_0
 *   for j = 0 .. m-1:
 *     w = A v_j;  for i = 0..j: h_ij = w.v_i, w -= h_ij v_i;  h_{j+1,j} = ||w||
 *     rotate column j by the earlier rotations, then zero h_{j+1,j} with a new
 *     one (c, s) = (h_jj, h_{j+1,j}) / hypot(h_jj, h_{j+1,j}); g_{j+1} = -s g_j,
 *     g_j = c g_j;  stop the cycle if |g_{j+1}| <= tau ||b||, the cap is
 *     reached or h_{j+1,j} = 0;  v_{j+1} = w / h_{j+1,j}
 *   solve the triangular R y = g over the columns used;  x += V y
 *
 * The triangular solve uses the columns built in the cycle (a cap in the
 * middle of a cycle still updates x).
 */
static int gmres_core(int64_t n, const int64_t *row_ptr, const int64_t *col, const double *val,
                      const double *b, double *x, double tau, int64_t max_iters, int64_t m,
                      orc_cg_result *res, double *hist, const double *d) {
    if (m < 1) m = 1;
    const size_t vb = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *V = (double *)malloc(vb * (size_t)(m + 1));
    double *w = (double *)malloc(vb);
    double *H = (double *)calloc((size_t)((m + 1) * m), sizeof(double));   /* H[i * m + j] */
    double *cs = (double *)malloc(sizeof(double) * (size_t)m);
    double *sn = (double *)malloc(sizeof(double) * (size_t)m);
    double *g = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *y = (double *)malloc(sizeof(double) * (size_t)m);
    double *y_n = (double *)malloc(vb);   /* M^{-1}-scaled work vector */
    int64_t k = 0;
    int reason = ORC_RUNNING;
    double resnorm = 0.0;
    const double bnorm = sqrt(dot(n, b, b));
    res->rhs_norm = bnorm;

    if (!isfinite(bnorm)) {
        reason = ORC_NON_FINITE;
        resnorm = bnorm;
        goto done;
    }
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        reason = ORC_CONVERGED;
        resnorm = 0.0;
        if (hist) hist[0] = 0.0;
        goto done;
    }
    while (reason == ORC_RUNNING) {
        orc_residual(n, row_ptr, col, val, b, x, V);
        const double beta = sqrt(dot(n, V, V));
        resnorm = beta;
        if (k == 0 && hist) hist[0] = beta;
        if (!isfinite(beta)) { reason = ORC_NON_FINITE; break; }
        if (beta <= tau * bnorm) { reason = ORC_CONVERGED; break; }
        if (k >= max_iters) { reason = ORC_MAX_ITERS; break; }
        for (int64_t i = 0; i < n; ++i) V[i] = V[i] / beta;
        for (int64_t i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int64_t used = 0;
        for (int64_t j = 0; j < m; ++j) {
            const double *vj = V + (size_t)j * (size_t)n;
            if (d) {   /* w = A M^{-1} v_j */
                for (int64_t t = 0; t < n; ++t) y_n[t] = vj[t] / d[t];
                orc_spmv(n, row_ptr, col, val, y_n, w);
            } else {
                orc_spmv(n, row_ptr, col, val, vj, w);
            }
            for (int64_t i = 0; i <= j; ++i) {
                const double *vi = V + (size_t)i * (size_t)n;
                const double h = dot(n, w, vi);
                H[i * m + j] = h;
                for (int64_t t = 0; t < n; ++t) w[t] = w[t] - h * vi[t];
            }
            const double hnext = sqrt(dot(n, w, w));
            for (int64_t i = 0; i < j; ++i) {
                const double a = H[i * m + j], c = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            const double a = H[j * m + j];
            const double d = hypot(a, hnext);
            if (d == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
            else { cs[j] = a / d; sn[j] = hnext / d; }
            H[j * m + j] = cs[j] * a + sn[j] * hnext;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k += 1;
            used = j + 1;
            resnorm = fabs(g[j + 1]);
            if (hist) hist[k] = resnorm;
            if (!isfinite(resnorm)) { reason = ORC_NON_FINITE; break; }
            if (resnorm <= tau * bnorm) { reason = ORC_CONVERGED; break; }
            if (k >= max_iters) { reason = ORC_MAX_ITERS; break; }
            if (hnext == 0.0) break;
            double *vn = V + (size_t)(j + 1) * (size_t)n;
            for (int64_t t = 0; t < n; ++t) vn[t] = w[t] / hnext;
        }
        if (reason == ORC_NON_FINITE) break;
        for (int64_t i = used - 1; i >= 0; --i) {
            double s = g[i];
            for (int64_t t = i + 1; t < used; ++t) s -= H[i * m + t] * y[t];
            y[i] = s / H[i * m + i];
        }
        if (d) {   /* x += M^{-1} (V y) */
            for (int64_t t = 0; t < n; ++t) y_n[t] = 0.0;
            for (int64_t i = 0; i < used; ++i) {
                const double *vi = V + (size_t)i * (size_t)n;
                for (int64_t t = 0; t < n; ++t) y_n[t] = y_n[t] + y[i] * vi[t];
            }
            for (int64_t t = 0; t < n; ++t) x[t] = x[t] + y_n[t] / d[t];
        } else {
            for (int64_t i = 0; i < used; ++i) {
                const double *vi = V + (size_t)i * (size_t)n;
                for (int64_t t = 0; t < n; ++t) x[t] = x[t] + y[i] * vi[t];
            }
        }
    }

done:
    res->iterations = k;
    res->stop_reason = reason;
    res->implicit_resnorm = resnorm;
    if (reason != ORC_NON_FINITE && n > 0) {
        orc_residual(n, row_ptr, col, val, b, x, w);
        res->true_resnorm = sqrt(dot(n, w, w));
    } else {
        res->true_resnorm = (n > 0) ? NAN : 0.0;
    }
    free(V); free(w); free(H); free(cs); free(sn); free(g); free(y); free(y_n);
    return reason;
}

int orc_gmres(int64_t n, const int64_t *row_ptr, const int64_t *col, const double *val,
              const double *b, double *x, double tau, int64_t max_iters, int64_t m,
              orc_cg_result *res, double *hist) {
    return gmres_core(n, row_ptr, col, val, b, x, tau, max_iters, m, res, hist, NULL);
}

int orc_gmres_jacobi(int64_t n, const int64_t *row_ptr, const int64_t *col, const double *val,
                     const double *b, double *x, double tau, int64_t max_iters, int64_t m,
                     orc_cg_result *res, double *hist) {
    double *d = NULL;
    if (!jacobi_diag_ok(n, row_ptr, col, val, b, x, res, &d)) return res->stop_reason;
    const int reason = gmres_core(n, row_ptr, col, val, b, x, tau, max_iters, m, res, hist, d);
    free(d);
    return reason;
}


/*
 * nnz-balanced row partition into P parts:
 *   split[j] = min { i in [0, n] : row_ptr[i] >= floor(j * nnz / P) },  j = 0..P-1
 *   split[P] = n
 * Part j owns rows [split[j], split[j+1]).
 */
void orc_partition(int64_t n, const int64_t *row_ptr, int64_t P, int64_t *split) {
    const int64_t nnz = row_ptr[n];
    int64_t i = 0;
    for (int64_t j = 0; j < P; ++j) {
        const int64_t target = (int64_t)(((__int128)j * nnz) / P);
        while (i < n && row_ptr[i] < target) ++i;
        split[j] = i;
    }
    split[P] = n;
}

/*
 * Gershgorin bound on the spectral condition number of a matrix whose rows
 * are strictly diagonally dominant with positive diagonal:
 *   kappa_G = max_i (a_ii + R_i) / min_i (a_ii - R_i),  R_i = sum_{j != i} |a_ij|.
 * Returns +inf when some row is not strictly dominant.
 */
double orc_gershgorin_kappa(int64_t n, const int64_t *row_ptr, const int64_t *col,
                            const double *val) {
    double hi = -INFINITY, lo = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0, R = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            if (col[k] == i) d += val[k];
            else R += fabs(val[k]);
        }
        if (d + R > hi) hi = d + R;
        if (d - R < lo) lo = d - R;
    }
    if (!(lo > 0.0)) return INFINITY;
    return hi / lo;
}
