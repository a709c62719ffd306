/*
 * Seeded synthetic inputs for the sparse Krylov solve (CPU side).
 *
 * This module builds inputs only: matrices, right-hand sides and instance
 * sizes.  It holds none of the solver's arithmetic and is the one piece of
 * code that both the HIP path and the FP64 oracle consume.
 *
 * Random numbers: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) used as a
 * counter-based generator.  For a (seed, stream, counter) triple
 *     K = mix64(seed * G + stream)
 *     h = mix64(K + (counter + 1) * G)          (all arithmetic mod 2^64)
 * where G = 0x9E3779B97F4A7C15 and mix64 is SplitMix64's output finaliser.
 * h is the (counter+1)-th SplitMix64 output of a generator seeded with K.
 *   uniform in [-1,1), FP64:  v = 2 * ((h >> 11) * 2^-53) - 1   (exact)
 *   uniform in [-1,1), FP32-exact: v = (h >> 40) * 2^-23 - 1    (exact in FP32)
 *
 * Streams: 0 off-diagonal matrix values, 1 randsym partner draws, 2 right-hand
 * side, 3 per-instance seeds, 4 per-instance sizes, 5 hub rows and their
 * lengths, 6 hub partner draws.
 *
 * Matrix patterns (the paper's test sets are SuiteSparse matrices with
 * dimension up to 1e6, density below 1%, and 0.6-41 nonzeros per row,
 * Section 6 and Table 2; these stand in for them):
 *   stencil7(N): 3-D N x N x N grid, row i = x + N*y + N*N*z couples to its
 *     +-1, +-N, +-N^2 neighbours; nnz = 7N^3 - 6N^2.  The undirected edge
 *     between i and its + neighbour in direction d (0:x,1:y,2:z) has id 3*i+d.
 *   randsym(n): row i draws 3 partners j uniform over [0,n) \ {i}; the pattern
 *     is symmetrised, sorted and merged.  Edge {i,j} has id min*n + max.
 *   powerlaw(n, hubs, lo, hi): randsym(n) plus `hubs` hub rows: hub h sits at
 *     row v(5, 2h) mod n and draws m_h partners (m_h log-uniform in [lo, hi]
 *     from v(5, 2h+1)), partner t uniform over [0,n) \ {hub} from stream 6,
 *     counter h * 2^32 + t; symmetrised and merged like randsym, so each hub
 *     row holds up to m_h + 7 entries and its partners one more each (the
 *     heavy-tailed row lengths of Table 2's circuit and mesh matrices).
 * Values: a_ij = a_ji = v(seed, 0, edge id); a_ii = sum_{j != i} |a_ij| + delta
 * accumulated in ascending column order in FP64, so A is symmetric and
 * strictly diagonally dominant with positive diagonal, hence SPD.
 * In the FP32-exact variant the off-diagonals use the FP32-exact draw and the
 * diagonal is rounded up to the next FP32 value, which keeps dominance.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GEN_GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t gen_hash(uint64_t seed, uint64_t stream, uint64_t ctr) {
    uint64_t k = mix64(seed * GEN_GOLDEN + stream);
    return mix64(k + (ctr + 1) * GEN_GOLDEN);
}

double gen_unif_f64(uint64_t seed, uint64_t stream, uint64_t ctr) {
    uint64_t h = gen_hash(seed, stream, ctr);
    double u = (double)(h >> 11) * 0x1.0p-53;
    return 2.0 * u - 1.0;
}

double gen_unif_f32x(uint64_t seed, uint64_t stream, uint64_t ctr) {
    uint64_t h = gen_hash(seed, stream, ctr);
    return (double)(int64_t)(h >> 40) * 0x1.0p-23 - 1.0;
}

static inline double offdiag(uint64_t seed, uint64_t edge, int f32x) {
    return f32x ? gen_unif_f32x(seed, 0, edge) : gen_unif_f64(seed, 0, edge);
}

/* Round a positive double up to the nearest FP32 value (returned as double). */
static double round_up_f32(double d) {
    float f = (float)d;
    if ((double)f < d) f = nextafterf(f, INFINITY);
    return (double)f;
}

int64_t gen_stencil7_nnz(int64_t N) {
    if (N <= 0) return 0;
    return 7 * N * N * N - 6 * N * N;
}

/*
 * Fill a stencil7 CSR matrix.  row_ptr has n+1 entries (n = N^3), col/val
 * have gen_stencil7_nnz(N) entries.  Rows are emitted in ascending column
 * order.  Returns 0, or -1 for N < 1.
 */
int gen_stencil7(int64_t N, uint64_t seed, double delta, int f32x,
                 int64_t *row_ptr, int32_t *col, double *val) {
    if (N < 1) return -1;
    const int64_t n = N * N * N, s1 = N, s2 = N * N;
    int64_t k = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t x = i % N, y = (i / N) % N, z = i / s2;
        int64_t cj[7];
        double cv[7];
        int m = 0, dpos = -1;
        /* ascending column order: -N^2, -N, -1, diag, +1, +N, +N^2 */
        if (z > 0)     { cj[m] = i - s2; cv[m] = offdiag(seed, 3 * (uint64_t)(i - s2) + 2, f32x); ++m; }
        if (y > 0)     { cj[m] = i - s1; cv[m] = offdiag(seed, 3 * (uint64_t)(i - s1) + 1, f32x); ++m; }
        if (x > 0)     { cj[m] = i - 1;  cv[m] = offdiag(seed, 3 * (uint64_t)(i - 1) + 0, f32x); ++m; }
        dpos = m; cj[m] = i; cv[m] = 0.0; ++m;
        if (x < N - 1) { cj[m] = i + 1;  cv[m] = offdiag(seed, 3 * (uint64_t)i + 0, f32x); ++m; }
        if (y < N - 1) { cj[m] = i + s1; cv[m] = offdiag(seed, 3 * (uint64_t)i + 1, f32x); ++m; }
        if (z < N - 1) { cj[m] = i + s2; cv[m] = offdiag(seed, 3 * (uint64_t)i + 2, f32x); ++m; }
        double d = 0.0;
        for (int t = 0; t < m; ++t)
            if (t != dpos) d += fabs(cv[t]);
        d += delta;
        cv[dpos] = f32x ? round_up_f32(d) : d;
        for (int t = 0; t < m; ++t) { col[k] = (int32_t)cj[t]; val[k] = cv[t]; ++k; }
        row_ptr[i + 1] = k;
    }
    return 0;
}

/* Entries of one row i of stencil7(N) (ascending columns) into cols/vals
 * (7 slots each); returns the count.  Same arithmetic as gen_stencil7. */
int gen_stencil7_row(int64_t N, uint64_t seed, double delta, int f32x, int64_t i, int64_t *cols, double *vals) {
    const int64_t s1 = N, s2 = N * N;
    const int64_t x = i % N, y = (i / N) % N, z = i / s2;
    int m = 0, dpos;
    if (z > 0)     { cols[m] = i - s2; vals[m] = offdiag(seed, 3 * (uint64_t)(i - s2) + 2, f32x); ++m; }
    if (y > 0)     { cols[m] = i - s1; vals[m] = offdiag(seed, 3 * (uint64_t)(i - s1) + 1, f32x); ++m; }
    if (x > 0)     { cols[m] = i - 1;  vals[m] = offdiag(seed, 3 * (uint64_t)(i - 1) + 0, f32x); ++m; }
    dpos = m; cols[m] = i; vals[m] = 0.0; ++m;
    if (x < N - 1) { cols[m] = i + 1;  vals[m] = offdiag(seed, 3 * (uint64_t)i + 0, f32x); ++m; }
    if (y < N - 1) { cols[m] = i + s1; vals[m] = offdiag(seed, 3 * (uint64_t)i + 1, f32x); ++m; }
    if (z < N - 1) { cols[m] = i + s2; vals[m] = offdiag(seed, 3 * (uint64_t)i + 2, f32x); ++m; }
    double d = 0.0;
    for (int t = 0; t < m; ++t)
        if (t != dpos) d += fabs(vals[t]);
    d += delta;
    vals[dpos] = f32x ? round_up_f32(d) : d;
    return m;
}

/* Rows [r0, r1) of stencil7(N) as a block: row_ptr (r1 - r0 + 1 entries,
 * starting at 0), column indices (global, ascending per row) and values, the
 * same entries gen_stencil7 emits for those rows.  col/val hold at least
 * 7 (r1 - r0) entries.  Returns the block's entry count, or -1 for bad
 * arguments. */
int64_t gen_stencil7_block(int64_t N, uint64_t seed, double delta, int f32x, int64_t r0, int64_t r1,
                           int64_t *row_ptr, int64_t *col, double *val) {
    if (N < 1 || r0 < 0 || r1 < r0 || r1 > N * N * N) return -1;
    int64_t k = 0;
    row_ptr[0] = 0;
    for (int64_t i = r0; i < r1; ++i) {
        k += gen_stencil7_row(N, seed, delta, f32x, i, col + k, val + k);
        row_ptr[i - r0 + 1] = k;
    }
    return k;
}

/*
 * stencil7_ns(N): the stencil7 pattern with every off-diagonal entry drawn on
 * its own (a_ij and a_ji independent, so A is nonsymmetric): entry (i, dir)
 * is uniform[-1,1) draw (seed, stream 16, 6 i + dir), dir = 0..5 for the
 * neighbours -N^2, -N, -1, +1, +N, +N^2.  Diagonal = sum of |off-diagonals|
 * of the row (ascending column order) + delta: strictly row diagonally
 * dominant.  Same sizes as stencil7.
 */
int gen_stencil7_ns(int64_t N, uint64_t seed, double delta, int64_t *row_ptr, int32_t *col, double *val) {
    if (N < 1) return -1;
    const int64_t n = N * N * N, s1 = N, s2 = N * N;
    int64_t k = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t x = i % N, y = (i / N) % N, z = i / s2;
        const uint64_t e0 = 6 * (uint64_t)i;
        int64_t cj[7];
        double cv[7];
        int m = 0, dpos = -1;
        if (z > 0)     { cj[m] = i - s2; cv[m] = gen_unif_f64(seed, 16, e0 + 0); ++m; }
        if (y > 0)     { cj[m] = i - s1; cv[m] = gen_unif_f64(seed, 16, e0 + 1); ++m; }
        if (x > 0)     { cj[m] = i - 1;  cv[m] = gen_unif_f64(seed, 16, e0 + 2); ++m; }
        dpos = m; cj[m] = i; cv[m] = 0.0; ++m;
        if (x < N - 1) { cj[m] = i + 1;  cv[m] = gen_unif_f64(seed, 16, e0 + 3); ++m; }
        if (y < N - 1) { cj[m] = i + s1; cv[m] = gen_unif_f64(seed, 16, e0 + 4); ++m; }
        if (z < N - 1) { cj[m] = i + s2; cv[m] = gen_unif_f64(seed, 16, e0 + 5); ++m; }
        double d = 0.0;
        for (int t = 0; t < m; ++t)
            if (t != dpos) d += fabs(cv[t]);
        cv[dpos] = d + delta;
        for (int t = 0; t < m; ++t) { col[k] = (int32_t)cj[t]; val[k] = cv[t]; ++k; }
        row_ptr[i + 1] = k;
    }
    return 0;
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/*
 * randsym(n): returns nnz (>= n), or -1 on bad arguments / -2 on allocation
 * failure.  row_ptr has n+1 entries; col/val must hold at least
 * gen_randsym_max_nnz(n, deg) entries.  Construction: count (histogram),
 * exclusive scan, scatter, per-row ascending sort, duplicate merge, then the
 * diagonal is inserted in its sorted position.
 */
int64_t gen_randsym_max_nnz(int64_t n, int deg) { return n + 2 * (int64_t)deg * n; }

/* Symmetric pattern from m directed draws (src[k], dst_of[k]) (both owned by
 * the caller); values and diagonal as described at the top. */
static int64_t build_sym(int64_t n, uint64_t seed, double delta, int f32x, int64_t m, const int64_t *src,
                         const int64_t *tgt, int64_t *row_ptr, int32_t *col, double *val) {
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *dst = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
    if (!cnt || !dst) { free(cnt); free(dst); return -2; }
    for (int64_t k = 0; k < m; ++k) { cnt[src[k] + 1]++; cnt[tgt[k] + 1]++; }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];          /* exclusive scan */
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!fill) { free(cnt); free(dst); return -2; }
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)n);
    for (int64_t k = 0; k < m; ++k) {
        const int64_t i = src[k], j = tgt[k];
        dst[fill[i]++] = j;
        dst[fill[j]++] = i;
    }
    free(fill);
    int64_t k = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t b = cnt[i], e = cnt[i + 1];
        qsort(dst + b, (size_t)(e - b), sizeof(int64_t), cmp_i64);
        /* merge duplicates, insert diagonal in sorted position */
        int64_t row_begin = k, dpos = -1;
        int64_t prev = -1;
        for (int64_t t = b; t < e; ++t) {
            int64_t j = dst[t];
            if (j == prev) continue;
            if (dpos < 0 && j > i) { dpos = k; col[k] = (int32_t)i; val[k] = 0.0; ++k; }
            uint64_t lo = (uint64_t)(i < j ? i : j), hi = (uint64_t)(i < j ? j : i);
            col[k] = (int32_t)j; val[k] = offdiag(seed, lo * (uint64_t)n + hi, f32x); ++k;
            prev = j;
        }
        if (dpos < 0) { dpos = k; col[k] = (int32_t)i; val[k] = 0.0; ++k; }
        double d = 0.0;
        for (int64_t t = row_begin; t < k; ++t)
            if (t != dpos) d += fabs(val[t]);
        d += delta;
        val[dpos] = f32x ? round_up_f32(d) : d;
        row_ptr[i + 1] = k;
    }
    free(cnt); free(dst);
    return k;
}

/* the deg * n partner draws of randsym(n) into src/tgt[0 .. deg*n) */
static void randsym_draws(int64_t n, uint64_t seed, int deg, int64_t *src, int64_t *tgt) {
    for (int64_t i = 0; i < n; ++i)
        for (int t = 0; t < deg; ++t) {
            uint64_t r = gen_hash(seed, 1, (uint64_t)deg * (uint64_t)i + (uint64_t)t);
            int64_t j = (int64_t)(r % (uint64_t)(n - 1));
            if (j >= i) j += 1;
            src[(int64_t)deg * i + t] = i;
            tgt[(int64_t)deg * i + t] = j;
        }
}

int64_t gen_randsym(int64_t n, uint64_t seed, double delta, int deg, int f32x,
                    int64_t *row_ptr, int32_t *col, double *val) {
    if (n < 1 || deg < 0) return -1;
    const int64_t m = (n >= 2) ? (int64_t)deg * n : 0; /* directed draws */
    int64_t *src = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t *tgt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    if (!src || !tgt) { free(src); free(tgt); return -2; }
    if (m > 0) randsym_draws(n, seed, deg, src, tgt);
    const int64_t k = build_sym(n, seed, delta, f32x, m, src, tgt, row_ptr, col, val);
    free(src); free(tgt);
    return k;
}

/* Hub h of powerlaw(n, ...): its row and its number of partner draws. */
void gen_powerlaw_hub(int64_t n, uint64_t seed, int64_t h, int64_t lo, int64_t hi, int64_t *row, int64_t *draws) {
    *row = (int64_t)(gen_hash(seed, 5, 2 * (uint64_t)h) % (uint64_t)n);
    const double u = 0.5 * (gen_unif_f64(seed, 5, 2 * (uint64_t)h + 1) + 1.0);   /* [0, 1) */
    int64_t m = (int64_t)llround(exp(log((double)lo) + u * (log((double)hi) - log((double)lo))));
    if (m < lo) m = lo;
    if (m > hi) m = hi;
    *draws = m;
}

int64_t gen_powerlaw_max_nnz(int64_t n, int deg, int64_t hubs, int64_t hi) {
    return n + 2 * (int64_t)deg * n + 2 * hubs * hi;
}

/* powerlaw(n, hubs, lo, hi): returns nnz, or -1 on bad arguments / -2 on
 * allocation failure; col/val must hold gen_powerlaw_max_nnz entries. */
int64_t gen_powerlaw(int64_t n, uint64_t seed, double delta, int deg, int64_t hubs, int64_t lo, int64_t hi, int f32x,
                     int64_t *row_ptr, int32_t *col, double *val) {
    if (n < 2 || deg < 0 || hubs < 0 || lo < 1 || hi < lo || hi > ((int64_t)1 << 32)) return -1;
    int64_t m = (int64_t)deg * n;
    for (int64_t h = 0; h < hubs; ++h) {
        int64_t r, d;
        gen_powerlaw_hub(n, seed, h, lo, hi, &r, &d);
        m += d;
    }
    int64_t *src = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t *tgt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    if (!src || !tgt) { free(src); free(tgt); return -2; }
    randsym_draws(n, seed, deg, src, tgt);
    int64_t k = (int64_t)deg * n;
    for (int64_t h = 0; h < hubs; ++h) {
        int64_t r, d;
        gen_powerlaw_hub(n, seed, h, lo, hi, &r, &d);
        for (int64_t t = 0; t < d; ++t) {
            uint64_t x = gen_hash(seed, 6, ((uint64_t)h << 32) + (uint64_t)t);
            int64_t j = (int64_t)(x % (uint64_t)(n - 1));
            if (j >= r) j += 1;
            src[k] = r;
            tgt[k] = j;
            ++k;
        }
    }
    const int64_t nnz = build_sym(n, seed, delta, f32x, m, src, tgt, row_ptr, col, val);
    free(src); free(tgt);
    return nnz;
}

/* Right-hand side: b_i = v(seed, 2, i) in [-1,1). */
void gen_rhs(int64_t n, uint64_t seed, double *b) {
    for (int64_t i = 0; i < n; ++i) b[i] = gen_unif_f64(seed, 2, (uint64_t)i);
}

/* Generic uniform vector on an arbitrary stream (used for SpMV inputs). */
void gen_vec(int64_t n, uint64_t seed, uint64_t stream, double *v) {
    for (int64_t i = 0; i < n; ++i) v[i] = gen_unif_f64(seed, stream, (uint64_t)i);
}

/*
 * Batched-serving instance table: n_i = round(exp(U[ln lo, ln hi])) with
 * U drawn from stream 4, and a per-instance matrix seed from stream 3.
 */
void gen_instances(int64_t count, uint64_t seed, double lo, double hi,
                   int64_t *sizes, uint64_t *seeds) {
    const double a = log(lo), b = log(hi);
    for (int64_t i = 0; i < count; ++i) {
        uint64_t h = gen_hash(seed, 4, (uint64_t)i);
        double u = (double)(h >> 11) * 0x1.0p-53;
        sizes[i] = (int64_t)llround(exp(a + (b - a) * u));
        seeds[i] = gen_hash(seed, 3, (uint64_t)i);
    }
}
