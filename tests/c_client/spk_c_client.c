/*
 * A plain C client of the spk C ABI: no Python, no torch.  It loads a CSR
 * system from binary files, copies it to the device with the HIP runtime,
 * runs spk_csr_check, an SpMV plan and a solve, and writes the product and
 * the solution back to files for the test to compare with the oracle.
 *
 *   spk_c_client DIR SOLVER PRECOND TAU MAX_ITERS
 *
 * DIR holds meta.txt ("n nnz"), row_ptr.i32, col.i32, val.f64, b.f64, x.f64
 * (the vector of the product); the client writes y.f64, sol.f64 and prints
 * one line "verdict iterations stop_reason rhs_norm true_resnorm".
 * SOLVER: 0 CG, 1 CGS, 2 GMRES; PRECOND: 0 none, 1 Jacobi.
 * SOLVER 9: the serving API instead of a plan: three requests on the same
 * matrix with right-hand sides b, b/2 and -b (mixed FP32 with FP64
 * refinement) submitted together, drained, and their solutions written to
 * sol.f64, sol_half.f64 and sol_neg.f64; the line printed is request 0's.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "spk.h"

static void *read_file(const char *dir, const char *name, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) { fprintf(stderr, "cannot open %s\n", path); exit(2); }
    void *p = malloc(bytes ? bytes : 1);
    if (bytes && fread(p, 1, bytes, f) != bytes) { fprintf(stderr, "short read %s\n", path); exit(2); }
    fclose(f);
    return p;
}

static void write_file(const char *dir, const char *name, const void *p, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(p, 1, bytes, f) != bytes) { fprintf(stderr, "cannot write %s\n", path); exit(2); }
    fclose(f);
}

static void *to_device(const void *h, size_t bytes) {
    void *d = NULL;
    if (hipMalloc(&d, bytes ? bytes : 16) != hipSuccess) { fprintf(stderr, "hipMalloc failed\n"); exit(3); }
    if (bytes && hipMemcpy(d, h, bytes, hipMemcpyHostToDevice) != hipSuccess) { fprintf(stderr, "H2D failed\n"); exit(3); }
    return d;
}

#define CHECK(call)                                                                     \
    do {                                                                                \
        spk_status s_ = (call);                                                         \
        if (s_ != SPK_OK) {                                                             \
            fprintf(stderr, "%s: %s (%s)\n", #call, spk_status_string(s_), spk_last_error(ctx)); \
            return 4;                                                                   \
        }                                                                               \
    } while (0)

int main(int argc, char **argv) {
    if (argc != 6) { fprintf(stderr, "usage: %s DIR SOLVER PRECOND TAU MAX_ITERS\n", argv[0]); return 1; }
    const char *dir = argv[1];
    long long n = 0, nnz = 0;
    {
        char path[4096];
        snprintf(path, sizeof path, "%s/meta.txt", dir);
        FILE *f = fopen(path, "r");
        if (!f || fscanf(f, "%lld %lld", &n, &nnz) != 2) { fprintf(stderr, "bad meta.txt\n"); return 2; }
        fclose(f);
    }
    int *rp = read_file(dir, "row_ptr.i32", sizeof(int) * (size_t)(n + 1));
    int *col = read_file(dir, "col.i32", sizeof(int) * (size_t)nnz);
    double *val = read_file(dir, "val.f64", sizeof(double) * (size_t)nnz);
    double *b = read_file(dir, "b.f64", sizeof(double) * (size_t)n);
    double *xv = read_file(dir, "x.f64", sizeof(double) * (size_t)n);

    spk_csr A;
    A.n_rows = n;
    A.n_cols = n;
    A.nnz = nnz;
    A.ptr_type = SPK_I32;
    A.idx_type = SPK_I32;
    A.val_type = SPK_F64;
    A.reserved = 0;
    A.row_ptr = to_device(rp, sizeof(int) * (size_t)(n + 1));
    A.col_idx = to_device(col, sizeof(int) * (size_t)nnz);
    A.values = to_device(val, sizeof(double) * (size_t)nnz);
    double *d_b = to_device(b, sizeof(double) * (size_t)n);
    double *d_xv = to_device(xv, sizeof(double) * (size_t)n);
    double *d_y = NULL, *d_x = NULL;
    if (hipMalloc((void **)&d_y, sizeof(double) * (size_t)n) != hipSuccess ||
        hipMalloc((void **)&d_x, sizeof(double) * (size_t)n) != hipSuccess ||
        hipMemset(d_x, 0, sizeof(double) * (size_t)n) != hipSuccess)
        return 3;

    spk_ctx ctx = NULL;
    if (spk_init(0, NULL, &ctx) != SPK_OK) { fprintf(stderr, "spk_init failed\n"); return 4; }
    int32_t verdict = -1;
    CHECK(spk_csr_check(ctx, &A, &verdict));

    spk_plan sp = NULL;
    CHECK(spk_plan_spmv(ctx, &A, &sp));
    CHECK(spk_execute_spmv(sp, d_xv, d_y));
    CHECK(spk_free(sp));

    spk_solver_cfg cfg;
    spk_solver_cfg_default(&cfg);
    const int solver = atoi(argv[2]);
    cfg.precond = atoi(argv[3]);
    cfg.reduction_factor = atof(argv[4]);
    cfg.max_iters = atoll(argv[5]);
    spk_log log;
    if (solver == 9) {
        /* serving: b, b/2 and -b (exact scalings) in one batch */
        double *bh = malloc(sizeof(double) * (size_t)n), *bn = malloc(sizeof(double) * (size_t)n);
        for (long long i = 0; i < n; ++i) {
            bh[i] = 0.5 * b[i];
            bn[i] = -b[i];
        }
        double *d_bh = to_device(bh, sizeof(double) * (size_t)n), *d_bn = to_device(bn, sizeof(double) * (size_t)n);
        double *d_xh = NULL, *d_xn = NULL;
        if (hipMalloc((void **)&d_xh, sizeof(double) * (size_t)n) != hipSuccess ||
            hipMalloc((void **)&d_xn, sizeof(double) * (size_t)n) != hipSuccess ||
            hipMemset(d_xh, 0, sizeof(double) * (size_t)n) != hipSuccess ||
            hipMemset(d_xn, 0, sizeof(double) * (size_t)n) != hipSuccess)
            return 3;
        cfg.precision = SPK_PREC_MIXED_FP32;
        spk_server srv = NULL;
        CHECK(spk_server_create(ctx, (size_t)1 << 30, 4, &cfg, &srv));
        uint64_t t[3];
        CHECK(spk_server_submit(srv, &A, d_b, d_x, &t[0]));
        CHECK(spk_server_submit(srv, &A, d_bh, d_xh, &t[1]));
        CHECK(spk_server_submit(srv, &A, d_bn, d_xn, &t[2]));
        CHECK(spk_server_drain(srv));
        for (int k = 2; k >= 0; --k) {   /* request 0 last, so log ends as its log */
            int32_t done = 0;
            int64_t lat = 0;
            CHECK(spk_server_poll(srv, t[k], &done, &log, &lat));
            if (!done) { fprintf(stderr, "request %d not done after drain\n", k); return 5; }
        }
        CHECK(spk_server_destroy(srv));
        double *h = malloc(sizeof(double) * (size_t)n);
        if (hipMemcpy(h, d_xh, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) return 3;
        write_file(dir, "sol_half.f64", h, sizeof(double) * (size_t)n);
        if (hipMemcpy(h, d_xn, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) return 3;
        write_file(dir, "sol_neg.f64", h, sizeof(double) * (size_t)n);
        hipFree(d_bh);
        hipFree(d_bn);
        hipFree(d_xh);
        hipFree(d_xn);
        free(h);
        free(bh);
        free(bn);
    } else {
        cfg.solver = solver;
        spk_plan pl = NULL;
        CHECK(spk_plan_solve(ctx, &A, &cfg, &pl));
        CHECK(spk_execute_solve(pl, d_b, d_x, &log));
        CHECK(spk_free(pl));
    }
    CHECK(spk_finalize(ctx));

    double *y = malloc(sizeof(double) * (size_t)n), *sol = malloc(sizeof(double) * (size_t)n);
    if (hipMemcpy(y, d_y, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(sol, d_x, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess)
        return 3;
    write_file(dir, "y.f64", y, sizeof(double) * (size_t)n);
    write_file(dir, "sol.f64", sol, sizeof(double) * (size_t)n);
    printf("%d %lld %d %.17g %.17g\n", verdict, (long long)log.iterations, log.stop_reason, log.rhs_norm,
           log.true_resnorm);
    hipFree((void *)A.row_ptr);
    hipFree((void *)A.col_idx);
    hipFree((void *)A.values);
    hipFree(d_b);
    hipFree(d_xv);
    hipFree(d_y);
    hipFree(d_x);
    free(rp); free(col); free(val); free(b); free(xv); free(y); free(sol);
    return 0;
}
