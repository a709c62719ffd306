// Host runtime behind the spk C ABI (include/spk.h): contexts, plans,
// validation, the SpMV autotuner, and the CG driver (host-loop or
// graph-replayed chunks of iterations with a convergence-rate-predicted
// chunk size).  All GPU work goes through the launchers in spk_kernels.hip.
#include "spk.h"
#include "spk_internal.h"
#include "spk_launch.h"
#include "spk_pool.h"

#include <algorithm>
#include <cstddef>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

using spk::CsrDev;
using spk::SolveState;
using spk::SpmvTune;

namespace {

struct TuneKey {
    int64_t n_rows, n_cols, nnz;
    int pt, it, vt;
    int use;     // TUNE_PLAIN or TUNE_CG
    int codes;   // the matrix has column codes
    int staged;  // values and columns are 16-byte aligned (the LDS tiles may run)
    int long_rows;    // rows longer than kLongRow (the kernels with the long-row pass run)
    bool operator<(const TuneKey &o) const {
        return std::tie(n_rows, n_cols, nnz, pt, it, vt, use, codes, staged, long_rows) <
               std::tie(o.n_rows, o.n_cols, o.nnz, o.pt, o.it, o.vt, o.use, o.codes, o.staged, o.long_rows);
    }
};

// What a tuning run times: the plain product y = A x, or the solvers' SpMV
// fused with the p.q partials (its register count, and so its residency,
// differs).
enum { TUNE_PLAIN = 0, TUNE_CG = 1, TUNE_FCG = 2 };

struct TuneResult {
    SpmvTune tune;
    double ms;
};

}  // namespace

struct spk_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream used only for graph capture
    int num_cu = 0;
    int wall_khz = 0;                   // wall_clock64() rate
    std::string err;
    unsigned *d_flags = nullptr;
    unsigned *h_flags = nullptr;        // pinned; [2], [3]: the pattern probe's words
    long long *d_probe = nullptr;       // pattern probe: offset table (kCodeSlots) and 4 words
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t ev_snap = nullptr;       // marks a state snapshot copy in the solve loops
    std::map<TuneKey, TuneResult> tune_cache;
    spk::DevicePool dpool;              // plan workspace cache
    spk::PinnedPool hpool;              // pinned status mirrors
    int live_plans = 0;
    // allocation-free solves: this device's scratch array (address looked up
    // at spk_init) and a pinned status mirror made at spk_init
    void *scratch = nullptr;
    hipError_t scratch_err = hipSuccess;
    SolveState *h_noalloc_st = nullptr;
};

struct spk_plan_s {
    spk_ctx ctx = nullptr;
    int kind = 0;                        // 0 = SpMV, 1 = solve
    CsrDev A{};
    spk_solver_cfg cfg{};
    SpmvTune tune{};
    int vec_grid = 1;
    int persist_grid = 0;                // cooperative grid of the persistent solve (0 = not used)
    unsigned *bar = nullptr;             // persistent grid-barrier words
    spk::PersistResult *persist_res = nullptr;   // persistent mixed solve: its result (device)
    spk_plan_info info{};
    double *r = nullptr, *p = nullptr, *q = nullptr, *partials = nullptr, *hist = nullptr;
    int algo = 0;                        // ALGO_CG / ALGO_CGS / ALGO_PCG
    double *rt = nullptr, *u = nullptr, *v = nullptr, *uh = nullptr;   // CGS
    double *dinv = nullptr;              // Jacobi: 1 / diag(A)
    void *coo_rp = nullptr;              // COO SpMV: derived row pointer (owned)
    void *codes_buf = nullptr;           // column codes: offset table + one byte per entry (owned)
    void *gm_V = nullptr, *gm_w = nullptr;   // GMRES basis and work vector (FP64, or FP32 in GMRES-IR)
    double *gm_part = nullptr;               // GMRES per-workgroup partials
    spk::GmresState *gm_st = nullptr;    // GMRES small arrays
    unsigned *diag_flag = nullptr;       // Jacobi: nonzero = unusable diagonal
    bool right_jacobi = false;           // CGS / GMRES on A M^{-1}, M = diag(A)
    bool bad_diag = false;               // right Jacobi: unusable diagonal (every solve breaks down)
    CsrDev A_orig{};                     // right Jacobi: the caller's matrix (A holds A M^{-1})
    double *scaled_vals = nullptr;       // right Jacobi: values of A M^{-1}
    int64_t hist_cap = 0;
    SolveState *st = nullptr;
    SolveState *h_st = nullptr;          // pinned mirror
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;   // (loop kind, iterations) -> graph
    // mixed precision: inner CG on A32 with FP32 vectors
    CsrDev A32{};
    SpmvTune tune32{};
    void *a32_vals = nullptr;            // owned rounded copy (null when A32 aliases A)
    float *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr;
    SolveState *st_in = nullptr, *h_st_in = nullptr;
    double *out_dev = nullptr, *h_out = nullptr;   // refinement norms (device / pinned)
    // fused CG loop (one launch per iteration): second buffers of r, p, q
    // (FP64, or FP32 for the inner solve), paired with r, p, q / r32, p32, q32
    bool fused = false;
    double *r_b = nullptr, *p_b = nullptr, *q_b = nullptr;
    float *r32_b = nullptr, *p32_b = nullptr, *q32_b = nullptr;
    int profiling = 0;                   // time every profiling-th dominant SpMV launch (0 = off)
    int64_t prof_seq = 0;                // dominant SpMV launches since the last collect
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
    std::vector<char> ev_ok;             // 0: the recorded launch found nothing to do (left out)
    size_t ev_used = 0;
    double prof_ms = 0.0;
    int64_t prof_count = 0;
};

namespace {

spk_status fail(spk_ctx ctx, spk_status code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

spk_status hip_fail(spk_ctx ctx, hipError_t e, const char *what) {
    const spk_status code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? SPK_ERR_OUT_OF_MEMORY
                                                                                         : SPK_ERR_DEVICE;
    return fail(ctx, code, std::string(what) + ": " + hipGetErrorString(e));
}

#define SPK_HIP(ctx, expr)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

bool valid_itype(int t) { return t == SPK_I32 || t == SPK_I64; }
bool valid_dtype(int t) { return t >= SPK_F64 && t <= SPK_BF16; }

// Host-side argument checks that need no device access.
spk_status check_csr_args(spk_ctx ctx, const spk_csr *A) {
    if (!A) return fail(ctx, SPK_ERR_INVALID_ARG, "null matrix descriptor");
    if (!valid_itype(A->ptr_type) || !valid_itype(A->idx_type))
        return fail(ctx, SPK_ERR_INVALID_ARG, "unknown index type");
    if (!valid_dtype(A->val_type)) return fail(ctx, SPK_ERR_INVALID_ARG, "unknown value type");
    if (A->n_rows < 0 || A->n_cols < 0 || A->nnz < 0) return SPK_OK;   // reported as a verdict
    if (!A->row_ptr) return fail(ctx, SPK_ERR_INVALID_ARG, "row_ptr is null");
    if (A->nnz > 0 && (!A->col_idx || !A->values)) return fail(ctx, SPK_ERR_INVALID_ARG, "col_idx/values null");
    return SPK_OK;
}

CsrDev to_dev(const spk_csr *A) {
    CsrDev d;
    d.n_rows = A->n_rows;
    d.n_cols = A->n_cols;
    d.nnz = A->nnz;
    d.ptr_t = A->ptr_type;
    d.idx_t = A->idx_type;
    d.val_t = A->val_type;
    d.rp = A->row_ptr;
    d.ci = A->col_idx;
    d.va = A->values;
    return d;
}

size_t vec_bytes(int val_t) { return val_t == SPK_F64 ? 8 : 4; }

// max_row (optional): the longest row's entry count (valid for a valid A).
spk_status gpu_verdict(spk_ctx ctx, const spk_csr *A, int32_t *verdict, int64_t *max_row = nullptr) {
    if (A->n_rows < 0 || A->n_cols < 0 || A->nnz < 0) {
        *verdict = SPK_CSR_BAD_SIZE;
        return SPK_OK;
    }
    const CsrDev d = to_dev(A);
    SPK_HIP(ctx, hipMemsetAsync(ctx->d_flags, 0, 2 * sizeof(unsigned), ctx->stream));
    SPK_HIP(ctx, spk::launch_validate(d, ctx->d_flags, ctx->num_cu * 4, ctx->stream));
    SPK_HIP(ctx, hipMemcpyAsync(ctx->h_flags, ctx->d_flags, 2 * sizeof(unsigned), hipMemcpyDeviceToHost, ctx->stream));
    SPK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const unsigned f = ctx->h_flags[0];
    if (max_row) *max_row = ctx->h_flags[1];
    int32_t v = SPK_CSR_OK;
    if (f & spk::VFLAG_BAD_FIRST) v = SPK_CSR_BAD_FIRST;
    else if (f & spk::VFLAG_DECREASING) v = SPK_CSR_DECREASING;
    else if (f & spk::VFLAG_BAD_LAST) v = SPK_CSR_BAD_LAST;
    else if (f & spk::VFLAG_BAD_COLUMN) v = SPK_CSR_BAD_COLUMN;
    if (v == SPK_CSR_OK && A->ptr_type == SPK_I32 && A->nnz > INT32_MAX) v = SPK_CSR_BAD_LAST;
    *verdict = v;
    return SPK_OK;
}

const char *verdict_name(int32_t v) {
    switch (v) {
        case SPK_CSR_BAD_SIZE: return "negative size";
        case SPK_CSR_BAD_FIRST: return "row_ptr[0] != 0";
        case SPK_CSR_DECREASING: return "row_ptr decreases";
        case SPK_CSR_BAD_LAST: return "row_ptr[n_rows] != nnz";
        case SPK_CSR_BAD_COLUMN: return "column index out of range";
        default: return "ok";
    }
}

// ------------------------------------------------------------------ tuning
int64_t num_tiles(int64_t n) { return (n + spk::kTileRows - 1) / spk::kTileRows; }

// The LDS tiling stages with 16-byte loads: values and col_idx must be 16-byte aligned.
bool stream_ok(const CsrDev &A) {
    return (reinterpret_cast<uintptr_t>(A.va) & 15) == 0 && (reinterpret_cast<uintptr_t>(A.ci) & 15) == 0;
}

// bpc <= 0: as many workgroups per CU as the occupancy calculator allows;
// otherwise bpc per CU (extra workgroups queue until a slot frees).
SpmvTune make_tune(spk_ctx ctx, const CsrDev &A, int kind, int lanes_log2, int remap, int nt, int pf, int bpc,
                   int codes = 0, int pack = 0) {
    SpmvTune t{kind, lanes_log2, 1, remap, nt, pf, 0};
    t.cus = ctx->num_cu;
    t.codes = kind == 0 && codes && A.codes;
    t.pack = t.codes && pack && A.rowpack;
    const int occ = spk::spmv_blocks_per_cu(A, t);
    const int use = (bpc <= 0) ? occ : std::min(bpc, 32);   // a forced count may oversubscribe
    t.bpc = use;
    int64_t g = static_cast<int64_t>(ctx->num_cu) * use;
    g = std::min<int64_t>(g, spk::kMaxGrid);
    g = std::min<int64_t>(g, std::max<int64_t>(num_tiles(A.n_rows), 1));
    t.grid = static_cast<int>(std::max<int64_t>(g, 1));
    return t;
}

SpmvTune heuristic_tune(spk_ctx ctx, const CsrDev &A) {
    const double mean = A.n_rows > 0 ? static_cast<double>(A.nnz) / A.n_rows : 0.0;
    if (mean <= 16.0 && stream_ok(A)) return make_tune(ctx, A, 0, 0, 0, 0, 1, 0, 1, 1);
    int l2 = 0;
    while ((1 << l2) < mean && l2 < 6) ++l2;
    return make_tune(ctx, A, 1, l2, 1, 0, 0, 0);
}

// Times each candidate and keeps the fastest.  x, y: device vectors of the
// plan's vector type (contents irrelevant for timing).  use = TUNE_CG times
// the solvers' fused SpMV with st (stop flag clear) and partials.
spk_status autotune(spk_ctx ctx, const CsrDev &A, const void *x, void *y, int use, SolveState *st,
                    double *partials, TuneResult *out, const void *fcg = nullptr) {
    const TuneKey key{A.n_rows, A.n_cols, A.nnz, A.ptr_t, A.idx_t, A.val_t, use, A.codes != nullptr, stream_ok(A),
                      A.max_row > spk::kLongRow};
    auto hit = ctx->tune_cache.find(key);
    if (hit != ctx->tune_cache.end()) {
        *out = hit->second;
        return SPK_OK;
    }
    std::vector<SpmvTune> cands;
    const double mean = A.n_rows > 0 ? static_cast<double>(A.nnz) / A.n_rows : 0.0;
    if (stream_ok(A) && mean <= 64.0) {
        // tile-to-XCD maps (XCD-blocked runs of k tiles, contiguous eighths,
        // round-robin) x matrix loads cached or non-temporal, at the
        // occupancy calculator's workgroups per CU.  Ordered by prior
        // preference: XCD-blocked tile orders (at equal time they move fewer
        // bytes: stencil7 N=215, 1.20 GB per product against 1.36 GB
        // round-robin), non-temporal matrix loads (both measured best in the
        // CG loop).  One workgroup per CU above the calculator's figure is
        // not a candidate: those workgroups queue behind the resident ones,
        // and although back-to-back timings (which find the matrix partly in
        // the Infinity Cache) sometimes favour it, in the CG loop it measured
        // 16% slower at C2 (190 against 164 us) and 33% slower for the FP32
        // inner product at C3 (129 against 97 us).
        for (int remap : {64, 256, 1, 0})
            for (int nt : {1, 0}) {
                cands.push_back(make_tune(ctx, A, 0, 0, remap, nt, 1, 0));
            }
    }
    for (int l2 = 0; l2 <= 6; ++l2) {
        const double L = static_cast<double>(1 << l2);
        if (L > 4.0 * std::max(mean, 1.0) && l2 > 0) break;
        cands.push_back(make_tune(ctx, A, 1, l2, 1, 0, 0, 0));
    }
    auto launch = [&](const SpmvTune &t) -> hipError_t {
        if (use == TUNE_PLAIN) return spk::launch_spmv(A, t, x, y, ctx->stream);
        if (use == TUNE_FCG) {
            // step 0 of the fused loop (st->base = 0, the stop flag clear and
            // st->x set by the caller): the same gathers, stores and partials
            // as every later step
            if (A.val_t == SPK_F64)
                return spk::launch_fcg_step(A, t, 0, *static_cast<const spk::FcgBufs<double> *>(fcg), st, partials,
                                            ctx->stream);
            return spk::launch_fcg_step32(A, t, 0, *static_cast<const spk::FcgBufs<float> *>(fcg), st, partials,
                                          ctx->stream);
        }
        if (A.val_t == SPK_F64)
            return spk::launch_cg_spmv_pq(A, t, static_cast<const double *>(x), static_cast<double *>(y), st,
                                          partials, ctx->stream);
        return spk::launch_cg_spmv_pq32(A, t, static_cast<const float *>(x), static_cast<float *>(y), st, partials,
                                        ctx->stream);
    };
    auto time_one = [&](const SpmvTune &t, double *per) -> hipError_t {
        hipError_t e = launch(t);   // warm-up
        if (e == hipSuccess) e = hipEventRecord(ctx->ev0, ctx->stream);
        const int reps = 5;
        for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch(t);
        if (e == hipSuccess) e = hipEventRecord(ctx->ev1, ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(ctx->ev1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
        *per = ms / reps;
        return e;
    };
    TuneResult best{cands[0], 1e30};
    for (const SpmvTune &t : cands) {
        double per = 0.0;
        SPK_HIP(ctx, time_one(t, &per));
        // a later candidate must be 3% faster to replace the best: near-ties
        // (within timing noise, which a profiler attached to the process
        // widens) resolve to the earlier candidate, so runs choose alike
        if (per < 0.97 * best.ms) best = TuneResult{t, per};
    }
    if (A.codes && best.tune.kind == 0) {
        // the best tile order and cache policy on one-byte column codes, with
        // packed row pointers (when built) and without, each at the coded
        // kernel's own occupancy figure (in order of preference: fewer bytes
        // first, a later candidate must be 3% faster); the plain indices must
        // be 3% faster than the best coded candidate to be kept
        const SpmvTune b = best.tune;
        TuneResult coded{b, 1e30};
        for (int pack : {1, 0}) {
            if (pack && !A.rowpack) continue;
            const SpmvTune c = make_tune(ctx, A, 0, 0, b.xcd_remap, b.nt, b.pf, 0, 1, pack);
            double per = 0.0;
            SPK_HIP(ctx, time_one(c, &per));
            if (per < 0.97 * coded.ms) coded = TuneResult{c, per};
        }
        if (!(best.ms < 0.97 * coded.ms)) best = coded;
    }
    ctx->tune_cache[key] = best;
    *out = best;
    return SPK_OK;
}

// SPK_SPMV_KERNEL forces a tiling (tests and sweeps use it): "stream" or
// "vector:<lanes>", optionally followed by ",key=value" with keys remap, nt,
// pf, bpc, codes, pack (e.g. "stream,pf=1,nt=1,remap=0,bpc=4,codes=0";
// codes and pack default to 1 when the matrix has codes / packed rows).
bool forced_tune(spk_ctx ctx, const CsrDev &A, SpmvTune *t) {
    const char *env = std::getenv("SPK_SPMV_KERNEL");
    if (!env || !*env) return false;
    std::string v(env);
    int kind = -1, l2 = 0, remap = INT_MIN, nt = 0, pf = 1, bpc = 0, codes = 1, pack = 1;
    size_t pos = 0;
    bool first = true;
    while (pos <= v.size()) {
        size_t comma = v.find(',', pos);
        if (comma == std::string::npos) comma = v.size();
        const std::string tok = v.substr(pos, comma - pos);
        if (first) {
            if (tok == "stream") kind = 0;
            else if (tok == "stream-noremap") { kind = 0; remap = 0; }
            else if (tok.rfind("vector:", 0) == 0) {
                kind = 1;
                const int lanes = std::atoi(tok.c_str() + 7);
                while ((1 << l2) < lanes && l2 < 6) ++l2;
            }
            first = false;
        } else {
            const size_t eq = tok.find('=');
            if (eq != std::string::npos) {
                const std::string k = tok.substr(0, eq);
                const int val = std::atoi(tok.c_str() + eq + 1);
                if (k == "remap") remap = val;
                else if (k == "nt") nt = val;
                else if (k == "pf") pf = val;
                else if (k == "bpc") bpc = val;
                else if (k == "codes") codes = val;
                else if (k == "pack") pack = val;
            }
        }
        pos = comma + 1;
    }
    if (kind < 0) return false;
    if (kind == 0 && !stream_ok(A)) kind = 1;
    if (remap < 0) remap = 1;   // unset (or negative): contiguous XCD eighths
    *t = make_tune(ctx, A, kind, l2, remap, nt, pf, bpc, codes, pack);
    return true;
}

spk_status choose_tune(spk_plan pl, const void *x, void *y, int use = TUNE_PLAIN, SolveState *st = nullptr,
                       const void *fcg = nullptr) {
    spk_ctx ctx = pl->ctx;
    const CsrDev &A = pl->A;
    if (A.n_rows == 0) {
        pl->tune = SpmvTune{0, 0, 1, 0, 0, 0, 0};
        pl->info.tuned = 0;
        return SPK_OK;
    }
    if (forced_tune(ctx, A, &pl->tune)) {
        pl->info.tuned = 0;
    } else if (A.nnz >= 100000) {
        TuneResult tr;
        spk_status s = autotune(ctx, A, x, y, use, st, pl->partials, &tr, fcg);
        if (s != SPK_OK) return s;
        pl->tune = tr.tune;
        pl->info.tuned = 1;
        pl->info.spmv_ms = tr.ms;
    } else {
        pl->tune = heuristic_tune(ctx, A);
        pl->info.tuned = 0;
    }
    pl->info.spmv_kernel = pl->tune.kind;
    pl->info.lanes = 1 << pl->tune.lanes_log2;
    pl->info.grid = pl->tune.grid;
    pl->info.xcd_remap = pl->tune.xcd_remap;
    pl->info.nontemporal = pl->tune.nt;
    pl->info.col_codes =
        (pl->tune.kind == 0 && pl->tune.codes && A.codes) ? ((pl->tune.pack && A.rowpack) ? 3 : 1) : 0;
    return SPK_OK;
}

// One-byte column codes for the LDS-tile SpMV (kernels k_code_*): built when
// the pattern has at most kCodeDict distinct column offsets c - i and the
// LDS tiling can stage them, for matrices of at least kCodeMinNnz entries
// (below that the plan-time build and its read-back cost more than a solve
// saves: 3 bytes per entry per product).  SPK_COL_CODES=0 turns them off,
// SPK_COL_CODES=1 builds them at any size.  A pattern without codes, or a
// failed allocation, leaves the plain indices in use.  With the codes come
// packed row pointers (per tile an int64 base, per row a uint16 offset:
// 2 bytes per row instead of 4 or 8) unless a row starts 65536 or more
// entries into its tile; SPK_ROW_PACK=0 keeps the plain row pointers.
constexpr int64_t kCodeMinNnz = int64_t(1) << 22;

spk_status build_codes(spk_plan pl) {
    spk_ctx ctx = pl->ctx;
    CsrDev &A = pl->A;
    const char *env = std::getenv("SPK_COL_CODES");
    if ((env && std::strcmp(env, "0") == 0) || A.nnz == 0 || A.n_rows == 0 || !stream_ok(A)) return SPK_OK;
    // a row longer than kLongRow entries holds more than 256 distinct
    // offsets unless it repeats a column; such matrices keep their indices,
    // so the coded kernels never need the long-row pass
    if (A.max_row > spk::kLongRow) return SPK_OK;
    if (!(env && std::strcmp(env, "1") == 0) && A.nnz < kCodeMinNnz) return SPK_OK;
    void *tab = nullptr, *buf = nullptr;
    const size_t bytes = spk::code_buffer_bytes(A.n_rows, A.nnz);
    if (ctx->dpool.get(sizeof(long long) * spk::kCodeSlots + 4 * sizeof(unsigned), &tab) != hipSuccess)
        return SPK_OK;
    if (ctx->dpool.get(bytes, &buf) != hipSuccess) {   // no room for codes: plain indices
        ctx->dpool.put(tab);
        return SPK_OK;
    }
    long long *table = static_cast<long long *>(tab);
    unsigned *words = reinterpret_cast<unsigned *>(table + spk::kCodeSlots);
    unsigned h[3] = {0, 0, 0};
    // a sample of the tiles first (every 8th and the last: structured
    // patterns repeat their offsets); if an entry's offset was missed, all
    // tiles.  Eight workgroups per CU (the most that fit) for the
    // latency-bound walks.
    const int grid = ctx->num_cu * 8;
    bool ok = true;
    for (int step : {8, 1}) {
        ok = spk::launch_code_build(A, step, table, words, buf, grid, ctx->stream) == hipSuccess &&
             hipMemcpyAsync(h, words, sizeof(h), hipMemcpyDeviceToHost, ctx->stream) == hipSuccess &&
             hipStreamSynchronize(ctx->stream) == hipSuccess;
        if (!ok || !(h[1] & 2u)) break;
    }
    ctx->dpool.put(tab);
    if (!ok) {
        ctx->dpool.put(buf);
        return fail(ctx, SPK_ERR_DEVICE, "column codes");
    }
    if (h[1] != 0 || h[0] < 1 || h[0] > static_cast<unsigned>(spk::kCodeDict)) {
        ctx->dpool.put(buf);
        return SPK_OK;
    }
    pl->codes_buf = buf;
    A.codes = static_cast<const char *>(buf) + sizeof(int64_t) * spk::kCodeDict;
    const char *pack = std::getenv("SPK_ROW_PACK");
    if (h[2] == 0 && !(pack && std::strcmp(pack, "0") == 0))
        A.rowpack = static_cast<const char *>(A.codes) + spk::code_bytes(A.nnz);
    return SPK_OK;
}

// ------------------------------------------------------------------ profiling events
// idx (optional): the recorded launch's event index, -1 when not sampled.
spk_status prof_begin(spk_plan pl, hipEvent_t *end_ev, int64_t *idx = nullptr) {
    *end_ev = nullptr;
    if (idx) *idx = -1;
    if (!pl->profiling) return SPK_OK;
    if (pl->prof_seq++ % pl->profiling != 0) return SPK_OK;   // not sampled
    if (pl->ev_used == pl->ev_pool.size()) {
        hipEvent_t a, b;
        SPK_HIP(pl->ctx, hipEventCreate(&a));
        SPK_HIP(pl->ctx, hipEventCreate(&b));
        pl->ev_pool.emplace_back(a, b);
        pl->ev_ok.push_back(1);
    }
    if (idx) *idx = static_cast<int64_t>(pl->ev_used);
    pl->ev_ok[pl->ev_used] = 1;
    auto &pr = pl->ev_pool[pl->ev_used++];
    SPK_HIP(pl->ctx, hipEventRecord(pr.first, pl->ctx->stream));
    *end_ev = pr.second;
    return SPK_OK;
}

spk_status prof_end(spk_plan pl, hipEvent_t end_ev) {
    if (end_ev) SPK_HIP(pl->ctx, hipEventRecord(end_ev, pl->ctx->stream));
    return SPK_OK;
}

// Accumulate the recorded launches among the first `useful` launches (stream
// already synchronised): launches 0, k, 2k, ... were recorded, k = profiling;
// recorded launches marked as having found nothing to do are left out.  A
// solve restarts the count; SpMV plans count across calls (keep_seq).
spk_status prof_collect(spk_plan pl, int64_t useful, bool keep_seq = false) {
    const int64_t k = std::max(pl->profiling, 1);
    const int64_t sampled = useful <= 0 ? 0 : 1 + (useful - 1) / k;
    const size_t n = std::min<size_t>(pl->ev_used, static_cast<size_t>(sampled));
    for (size_t i = 0; i < n; ++i) {
        if (!pl->ev_ok[i]) continue;
        float ms = 0.f;
        SPK_HIP(pl->ctx, hipEventElapsedTime(&ms, pl->ev_pool[i].first, pl->ev_pool[i].second));
        pl->prof_ms += ms;
        pl->prof_count += 1;
    }
    pl->ev_used = 0;
    if (!keep_seq) pl->prof_seq = 0;
    return SPK_OK;
}

// ------------------------------------------------------------------ CG driver
// Loop kinds: FP64 CG on A, FP32 inner CG on A32 (mixed precision), FP64
// CGS, FP64 Jacobi-preconditioned CG.
enum { LOOP_FP64 = 0, LOOP_FP32 = 1, LOOP_CGS = 2, LOOP_PCG = 3 };
enum { ALGO_CG = 0, ALGO_CGS = 1, ALGO_PCG = 2, ALGO_GMRES = 3 };

// The fused loop (one launch per CG iteration, or one grid barrier per
// iteration in the persistent mode) runs CG in FP64 and the CG inner solve of
// the mixed precisions for small systems, and always in the persistent mode.
// Measured (ms per solve, fused / three launches): stencil7 n = 97,336:
// 0.65 / 0.74; n = 343,000: 1.18 / 1.14 (the three vectors the fused step
// gathers per entry cost more than the two launches it saves; 16% slower at
// n = 9.9e6); randsym n = 16,000: 0.62 / 0.66, n = 50,000: 0.67 / 0.68,
// n = 131,072: 1.09 / 0.84 (on a random pattern each gathered vector is a
// random read of its own).  So: up to kFusedMaxRowsAny rows always; up to
// kFusedMaxRows when the pattern is banded (pattern_regular); never above.
// SPK_CG_FUSED=1 / 0 forces it on / off (0 also rules out the persistent
// mode).
constexpr int64_t kFusedMaxRows = int64_t(1) << 17;
constexpr int64_t kFusedMaxRowsAny = int64_t(1) << 16;

// Whether the choice depends on the pattern (pattern_regular must be asked).
bool fused_needs_pattern(const spk_solver_cfg &cfg, int64_t n) {
    if (cfg.solver != SPK_SOLVER_CG || cfg.precond != SPK_PRECOND_NONE || std::getenv("SPK_CG_FUSED")) return false;
    return cfg.exec_mode != SPK_EXEC_PERSISTENT && n > kFusedMaxRowsAny && n <= kFusedMaxRows;
}

bool fused_loop(const spk_solver_cfg &cfg, int64_t n, bool regular) {
    if (cfg.solver != SPK_SOLVER_CG || cfg.precond != SPK_PRECOND_NONE) return false;
    const char *env = std::getenv("SPK_CG_FUSED");
    if (env && std::strcmp(env, "0") == 0) return false;
    if (env && std::strcmp(env, "1") == 0) return true;
    return n <= kFusedMaxRowsAny || (n <= kFusedMaxRows && regular) || cfg.exec_mode == SPK_EXEC_PERSISTENT;
}

// Whether valid A's pattern is banded: the row tiles sampled (every eighth
// and the last) hold at most kCodeDict distinct column offsets c - i.
spk_status pattern_regular(spk_ctx ctx, const CsrDev &A, bool *regular) {
    *regular = true;
    if (A.n_rows == 0 || A.nnz == 0) return SPK_OK;
    long long *table = ctx->d_probe;
    unsigned *words = reinterpret_cast<unsigned *>(table + spk::kCodeSlots);
    SPK_HIP(ctx, spk::launch_pattern_probe(A, 8, table, words, ctx->num_cu * 8, ctx->stream));
    SPK_HIP(ctx, hipMemcpyAsync(ctx->h_flags + 2, words, 2 * sizeof(unsigned), hipMemcpyDeviceToHost, ctx->stream));
    SPK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *regular = ctx->h_flags[3] == 0 && ctx->h_flags[2] <= static_cast<unsigned>(spk::kCodeDict);
    return SPK_OK;
}

// st->x := ptr (the tuner's runs of the fused step write through st->x).
spk_status set_state_x(spk_ctx ctx, SolveState *st, void *ptr) {
    void *v = ptr;
    SPK_HIP(ctx, hipMemcpyAsync(reinterpret_cast<char *>(st) + offsetof(SolveState, x), &v, sizeof(v),
                                hipMemcpyHostToDevice, ctx->stream));
    SPK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return SPK_OK;
}

spk::FcgBufs<double> fcg64(const spk_plan_s *pl) { return {{pl->r, pl->r_b}, {pl->p, pl->p_b}, {pl->q, pl->q_b}}; }
spk::FcgBufs<float> fcg32(const spk_plan_s *pl) {
    return {{pl->r32, pl->r32_b}, {pl->p32, pl->p32_b}, {pl->q32, pl->q32_b}};
}

// Iteration j of a chunk: q = A p with p.q partials; alpha and r -= alpha q
// with r.r partials; x += alpha p, the stop test and p = r + beta p.  A chunk
// of `count` iterations ends by advancing the base.
spk_status launch_iterations(spk_plan pl, int kind, int count, hipStream_t s, bool with_prof) {
    spk_ctx ctx = pl->ctx;
    const int64_t n = pl->A.n_rows;
    hipEvent_t e = nullptr;
    auto pb = [&]() { return with_prof ? prof_begin(pl, &e) : SPK_OK; };
    auto pe = [&]() { return with_prof ? prof_end(pl, e) : SPK_OK; };
    spk_status st = SPK_OK;
    for (int i = 0; i < count; ++i) {
        if (kind == LOOP_CGS) {
            SPK_HIP(ctx, spk::launch_cgs_dir(n, pl->vec_grid, pl->tune.grid, i, pl->r, pl->u, pl->p, pl->q, pl->st,
                                             pl->partials, s));
            if ((st = pb()) != SPK_OK) return st;
            SPK_HIP(ctx, spk::launch_cgs_spmv_v(pl->A, pl->tune, pl->p, pl->v, pl->rt, pl->st, pl->partials, s));
            if ((st = pe()) != SPK_OK) return st;
            SPK_HIP(ctx, spk::launch_cgs_update(n, pl->vec_grid, pl->tune.grid, i, pl->u, pl->v, pl->q, pl->uh,
                                                pl->st, pl->partials, s));
            if ((st = pb()) != SPK_OK) return st;
            SPK_HIP(ctx, spk::launch_cgs_spmv_r(pl->A, pl->tune, pl->uh, pl->r, pl->rt, pl->st, pl->partials, s));
            if ((st = pe()) != SPK_OK) return st;
            continue;
        }
        if (pl->fused && (kind == LOOP_FP64 || kind == LOOP_FP32)) {
            if ((st = pb()) != SPK_OK) return st;
            if (kind == LOOP_FP64)
                SPK_HIP(ctx, spk::launch_fcg_step(pl->A, pl->tune, i, fcg64(pl), pl->st, pl->partials, s));
            else
                SPK_HIP(ctx, spk::launch_fcg_step32(pl->A32, pl->tune32, i, fcg32(pl), pl->st_in, pl->partials, s));
            if ((st = pe()) != SPK_OK) return st;
            continue;
        }
        if ((st = pb()) != SPK_OK) return st;
        if (kind == LOOP_FP32)
            SPK_HIP(ctx, spk::launch_cg_spmv_pq32(pl->A32, pl->tune32, pl->p32, pl->q32, pl->st_in, pl->partials, s));
        else
            SPK_HIP(ctx, spk::launch_cg_spmv_pq(pl->A, pl->tune, pl->p, pl->q, pl->st, pl->partials, s));
        if ((st = pe()) != SPK_OK) return st;
        if (kind == LOOP_FP64) {
            SPK_HIP(ctx, spk::launch_cg_update(n, pl->vec_grid, pl->tune.grid, i, pl->r, pl->q, pl->st, pl->partials, s));
            SPK_HIP(ctx, spk::launch_cg_pupdate(n, pl->vec_grid, i, pl->r, pl->p, pl->st, pl->partials, s));
        } else if (kind == LOOP_PCG) {
            SPK_HIP(ctx, spk::launch_pcg_update(n, pl->vec_grid, pl->tune.grid, i, pl->r, pl->q, pl->dinv, pl->st,
                                                pl->partials, s));
            SPK_HIP(ctx, spk::launch_pcg_pupdate(n, pl->vec_grid, i, pl->r, pl->dinv, pl->p, pl->st, pl->partials, s));
        } else {
            SPK_HIP(ctx, spk::launch_cg_update32(n, pl->vec_grid, pl->tune32.grid, i, pl->r32, pl->q32, pl->st_in,
                                                 pl->partials, s));
            SPK_HIP(ctx, spk::launch_cg_pupdate32(n, pl->vec_grid, i, pl->r32, pl->p32, pl->st_in, pl->partials, s));
        }
    }
    if (kind == LOOP_CGS)
        SPK_HIP(ctx, spk::launch_cgs_check(pl->st, pl->partials, pl->tune.grid, count, s));
    else
        SPK_HIP(ctx, spk::launch_cg_chunk_end(kind == LOOP_FP32 ? pl->st_in : pl->st, count, s));
    return SPK_OK;
}

spk_status graph_for(spk_plan pl, int kind, int count, hipGraphExec_t *out) {
    auto it = pl->graphs.find({kind, count});
    if (it != pl->graphs.end()) {
        *out = it->second;
        return SPK_OK;
    }
    spk_ctx ctx = pl->ctx;
    hipGraph_t g = nullptr;
    SPK_HIP(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    spk_status s = launch_iterations(pl, kind, count, ctx->cap_stream, false);
    hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
    if (s != SPK_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipGraphInstantiate");
    pl->graphs[{kind, count}] = exec;
    *out = exec;
    return SPK_OK;
}

spk_status run_chunk(spk_plan pl, int kind, int count, bool graph) {
    if (!graph) return launch_iterations(pl, kind, count, pl->ctx->stream, pl->profiling != 0);
    // binary decomposition into cached power-of-two graphs
    for (int bit = 1 << 10; bit >= 1; bit >>= 1) {
        while (count >= bit) {
            hipGraphExec_t ex = nullptr;
            spk_status s = graph_for(pl, kind, bit, &ex);
            if (s != SPK_OK) return s;
            SPK_HIP(pl->ctx, hipGraphLaunch(ex, pl->ctx->stream));
            count -= bit;
        }
    }
    return SPK_OK;
}

spk_status pull(spk_ctx ctx, void *host, const void *dev, size_t bytes) {
    SPK_HIP(ctx, hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
    SPK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return SPK_OK;
}

// Next chunk length from the observed residual decay (a scheduling guess only;
// kernels become no-ops once the device-side stop flag is set).
int next_chunk(int prev, int64_t k0, double r0, int64_t k1, double r1, double thresh, int64_t left) {
    int next = std::min(2 * prev, 256);
    if (k1 > k0 && r0 > 0.0 && r1 > 0.0 && thresh > 0.0 && r1 < r0) {
        const double rate = std::pow(r1 / r0, 1.0 / static_cast<double>(k1 - k0));
        if (rate < 1.0 && rate > 0.0) {
            const double rem = std::log(thresh / r1) / std::log(rate);
            if (std::isfinite(rem)) next = static_cast<int>(std::ceil(rem * 1.15)) + 2;
        }
    }
    next = std::max(next, 1);
    next = std::min<int64_t>(next, std::max<int64_t>(left, 1));
    return std::min(next, 1024);
}

// Run CG iterations of one loop kind until the device-side state stops.
// The state must already be initialised (init / refinement kernels).  The
// host reads the state from a snapshot copy queued after the chunks launched
// so far, and queues the next chunk before waiting for it, so the device is
// never idle while the host decides: chunk lengths follow the observed
// residual decay, less the chunk already in flight, and launches past
// convergence return at once.
spk_status run_loop(spk_plan pl, int kind, int64_t max_iters, bool graph) {
    spk_ctx ctx = pl->ctx;
    SolveState *st = kind == LOOP_FP32 ? pl->st_in : pl->st;
    SolveState *h = kind == LOOP_FP32 ? pl->h_st_in : pl->h_st;
    const int cfg_chunk = pl->cfg.chunk_iters;
    auto snapshot = [&]() -> spk_status {
        SPK_HIP(ctx, hipMemcpyAsync(h, st, sizeof(SolveState), hipMemcpyDeviceToHost, ctx->stream));
        SPK_HIP(ctx, hipEventRecord(ctx->ev_snap, ctx->stream));
        return SPK_OK;
    };
    auto wait = [&]() -> spk_status {
        SPK_HIP(ctx, hipEventSynchronize(ctx->ev_snap));
        return SPK_OK;
    };
    spk_status s = snapshot();   // the state before the first chunk
    if (s != SPK_OK) return s;
    int inflight = static_cast<int>(std::max<int64_t>(0, std::min<int64_t>(cfg_chunk > 0 ? cfg_chunk : 8, max_iters)));
    if (inflight > 0 && (s = run_chunk(pl, kind, inflight, graph)) != SPK_OK) return s;
    if ((s = wait()) != SPK_OK) return s;
    if (h->stop != spk::STOP_RUNNING) return SPK_OK;   // the queued chunk's launches return at once
    int64_t covered = 0;   // iterations the next snapshot follows
    int64_t k_prev = h->iter;
    double r_prev = h->resnorm > 0.0 ? h->resnorm : 1.0;
    // before the first rate is known the speculative chunk is short: it only
    // has to outlast the host's read of the first snapshot
    int guess = cfg_chunk > 0 ? cfg_chunk : 2;
    while (true) {
        covered += inflight;
        if ((s = snapshot()) != SPK_OK) return s;
        // launches past max_iters: the fused loop decides its stop one
        // launch late, and the decision itself takes a launch
        const int64_t left = max_iters + 2 - covered;
        const int next = left > 0 ? static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(guess, left))) : 0;
        if (next > 0 && (s = run_chunk(pl, kind, next, graph)) != SPK_OK) return s;
        if ((s = wait()) != SPK_OK) return s;
        if (h->stop != spk::STOP_RUNNING) break;
        if (next == 0) return fail(ctx, SPK_ERR_INTERNAL, "iteration cap passed without stop");
        if (cfg_chunk > 0) {
            guess = cfg_chunk;
        } else {
            const int rem = next_chunk(std::max(inflight, 1), k_prev, r_prev, h->iter, h->resnorm, h->thresh,
                                       max_iters - h->iter);
            guess = std::max(rem - next, 1);
        }
        k_prev = h->iter;
        r_prev = h->resnorm;
        inflight = next;
    }
    return SPK_OK;
}

// Hand a plan's workspace back to the context pools (stream already idle).
void release_workspace(spk_plan pl) {
    spk_ctx ctx = pl->ctx;
    ctx->dpool.put(pl->r);
    ctx->dpool.put(pl->p);
    ctx->dpool.put(pl->q);
    ctx->dpool.put(pl->partials);
    ctx->dpool.put(pl->hist);
    ctx->dpool.put(pl->st);
    ctx->hpool.put(pl->h_st);
    ctx->dpool.put(pl->a32_vals);
    ctx->dpool.put(pl->r32);
    ctx->dpool.put(pl->p32);
    ctx->dpool.put(pl->q32);
    ctx->dpool.put(pl->d32);
    ctx->dpool.put(pl->st_in);
    ctx->hpool.put(pl->h_st_in);
    ctx->dpool.put(pl->out_dev);
    ctx->hpool.put(pl->h_out);
    ctx->dpool.put(pl->bar);
    ctx->dpool.put(pl->persist_res);
    pl->persist_res = nullptr;
    ctx->dpool.put(pl->rt);
    ctx->dpool.put(pl->u);
    ctx->dpool.put(pl->v);
    ctx->dpool.put(pl->uh);
    ctx->dpool.put(pl->dinv);
    ctx->dpool.put(pl->diag_flag);
    ctx->dpool.put(pl->coo_rp);
    ctx->dpool.put(pl->codes_buf);
    pl->codes_buf = nullptr;
    ctx->dpool.put(pl->scaled_vals);
    pl->scaled_vals = nullptr;
    ctx->dpool.put(pl->gm_V);
    ctx->dpool.put(pl->gm_w);
    ctx->dpool.put(pl->gm_part);
    ctx->dpool.put(pl->gm_st);
    ctx->dpool.put(pl->r_b);
    ctx->dpool.put(pl->p_b);
    ctx->dpool.put(pl->q_b);
    ctx->dpool.put(pl->r32_b);
    ctx->dpool.put(pl->p32_b);
    ctx->dpool.put(pl->q32_b);
    pl->r_b = pl->p_b = pl->q_b = nullptr;
    pl->r32_b = pl->p32_b = pl->q32_b = nullptr;
    pl->coo_rp = nullptr;
    pl->gm_V = pl->gm_w = pl->gm_part = nullptr;
    pl->gm_st = nullptr;
    pl->rt = pl->u = pl->v = pl->uh = pl->dinv = nullptr;
    pl->diag_flag = nullptr;
    pl->bar = nullptr;
    pl->r = pl->p = pl->q = pl->partials = pl->hist = nullptr;
    pl->st = pl->h_st = pl->st_in = pl->h_st_in = nullptr;
    pl->a32_vals = nullptr;
    pl->r32 = pl->p32 = pl->q32 = pl->d32 = nullptr;
    pl->out_dev = pl->h_out = nullptr;
}

}  // namespace

namespace spk {
int ctx_device(const spk_ctx_s *ctx) { return ctx ? ctx->device : 0; }
}  // namespace spk

// ==================================================================== C ABI
extern "C" {

void spk_solver_cfg_default(spk_solver_cfg *cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->solver = SPK_SOLVER_CG;
    cfg->precision = SPK_PREC_FP64;
    cfg->baseline = SPK_BASELINE_RHS_NORM;
    cfg->precond = SPK_PRECOND_NONE;
    cfg->max_iters = 1000;
    cfg->reduction_factor = 1e-6;
    cfg->exec_mode = SPK_EXEC_AUTO;
    cfg->chunk_iters = 0;
    cfg->record_history = 0;
    cfg->true_residual = 1;
    cfg->inner_reduction = 1e-4;
    cfg->max_outer = 50;
    cfg->krylov_dim = 30;
}

const char *spk_status_string(spk_status s) {
    switch (s) {
        case SPK_OK: return "SPK_OK";
        case SPK_ERR_INVALID_ARG: return "SPK_ERR_INVALID_ARG";
        case SPK_ERR_UNSUPPORTED: return "SPK_ERR_UNSUPPORTED";
        case SPK_ERR_OUT_OF_MEMORY: return "SPK_ERR_OUT_OF_MEMORY";
        case SPK_ERR_BUDGET: return "SPK_ERR_BUDGET";
        case SPK_ERR_DEVICE: return "SPK_ERR_DEVICE";
        case SPK_ERR_INTERNAL: return "SPK_ERR_INTERNAL";
        default: return "SPK_UNKNOWN_STATUS";
    }
}

const char *spk_last_error(spk_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

spk_status spk_init(int device_id, void *hip_stream, spk_ctx *out) {
    if (!out) return SPK_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device_id < 0 || device_id >= count) return SPK_ERR_INVALID_ARG;
    if (hipSetDevice(device_id) != hipSuccess) return SPK_ERR_DEVICE;
    spk_ctx ctx = new spk_ctx_s();
    ctx->device = device_id;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device_id) != hipSuccess) {
        delete ctx;
        return SPK_ERR_DEVICE;
    }
    ctx->num_cu = prop.multiProcessorCount;
    if (hipDeviceGetAttribute(&ctx->wall_khz, hipDeviceAttributeWallClockRate, device_id) != hipSuccess ||
        ctx->wall_khz <= 0)
        ctx->wall_khz = 100000;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) ctx->dpool.set_cap(total_b / 4);
    ctx->hpool.set_cap(size_t(16) << 20);
    if (hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc(&ctx->d_flags, 2 * sizeof(unsigned)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&ctx->h_flags), 4 * sizeof(unsigned), hipHostMallocDefault) !=
            hipSuccess ||
        hipMalloc(&ctx->d_probe, sizeof(long long) * spk::kCodeSlots + 4 * sizeof(unsigned)) != hipSuccess ||
        hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_snap, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&ctx->h_noalloc_st), sizeof(SolveState), hipHostMallocDefault) !=
            hipSuccess) {
        spk_finalize(ctx);
        return SPK_ERR_DEVICE;
    }
    // the scratch array's device address on this device (kept per device); a
    // failed lookup only disables spk_solve_noalloc
    ctx->scratch_err = spk::noalloc_scratch_setup(device_id, &ctx->scratch);
    *out = ctx;
    return SPK_OK;
}

spk_status spk_finalize(spk_ctx ctx) {
    if (!ctx) return SPK_OK;
    if (ctx->live_plans > 0) return fail(ctx, SPK_ERR_INVALID_ARG, "context still has live plans");
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    ctx->dpool.trim();
    ctx->hpool.trim();
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->d_flags) (void)hipFree(ctx->d_flags);
    if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
    if (ctx->d_probe) (void)hipFree(ctx->d_probe);
    if (ctx->h_noalloc_st) (void)hipHostFree(ctx->h_noalloc_st);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->ev_snap) (void)hipEventDestroy(ctx->ev_snap);
    delete ctx;
    return SPK_OK;
}

spk_status spk_csr_check(spk_ctx ctx, const spk_csr *A, int32_t *verdict) {
    if (!ctx || !verdict) return SPK_ERR_INVALID_ARG;
    SPK_HIP(ctx, hipSetDevice(ctx->device));
    spk_status s = check_csr_args(ctx, A);
    if (s != SPK_OK) return s;
    return gpu_verdict(ctx, A, verdict);
}

spk_status spk_partition(spk_ctx ctx, const spk_csr *A, int64_t parts, int64_t *split_dev) {
    if (!ctx || !split_dev) return SPK_ERR_INVALID_ARG;
    if (parts < 1 || parts > (int64_t(1) << 31)) return fail(ctx, SPK_ERR_INVALID_ARG, "parts out of range");
    spk_status s = check_csr_args(ctx, A);
    if (s != SPK_OK) return s;
    if (A->n_rows < 0) return fail(ctx, SPK_ERR_INVALID_ARG, "negative size");
    SPK_HIP(ctx, hipSetDevice(ctx->device));
    SPK_HIP(ctx, spk::launch_partition(to_dev(A), parts, split_dev, ctx->stream));
    SPK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return SPK_OK;
}

static spk_status plan_common(spk_ctx ctx, const spk_csr *A, spk_plan *out, int64_t *max_row) {
    if (!ctx || !out) return SPK_ERR_INVALID_ARG;
    *out = nullptr;
    SPK_HIP(ctx, hipSetDevice(ctx->device));
    spk_status s = check_csr_args(ctx, A);
    if (s != SPK_OK) return s;
    int32_t verdict = 0;
    s = gpu_verdict(ctx, A, &verdict, max_row);
    if (s != SPK_OK) return s;
    // SPK_LONG_ROWS=0: every row summed by one lane, however long (comparisons)
    const char *lr = std::getenv("SPK_LONG_ROWS");
    if (max_row && lr && std::strcmp(lr, "0") == 0) *max_row = 0;
    if (verdict != SPK_CSR_OK) return fail(ctx, SPK_ERR_INVALID_ARG, std::string("malformed CSR: ") + verdict_name(verdict));
    return SPK_OK;
}

// Tune and finish an SpMV plan whose matrix view is already set.
static spk_status finish_spmv_plan(spk_ctx ctx, spk_plan pl, const spk_csr *A, spk_plan *out);

spk_status spk_plan_spmv(spk_ctx ctx, const spk_csr *A, spk_plan *out) {
    int64_t max_row = 0;
    spk_status s = plan_common(ctx, A, out, &max_row);
    if (s != SPK_OK) return s;
    spk_plan pl = new spk_plan_s();
    pl->ctx = ctx;
    pl->kind = 0;
    pl->A = to_dev(A);
    pl->A.max_row = max_row;
    return finish_spmv_plan(ctx, pl, A, out);
}

static spk_status coo_args(spk_ctx ctx, const spk_coo *A) {
    if (!A) return fail(ctx, SPK_ERR_INVALID_ARG, "null matrix descriptor");
    if (!valid_itype(A->idx_type)) return fail(ctx, SPK_ERR_INVALID_ARG, "unknown index type");
    if (!valid_dtype(A->val_type)) return fail(ctx, SPK_ERR_INVALID_ARG, "unknown value type");
    if (A->nnz > 0 && (!A->row_idx || !A->col_idx || !A->values))
        return fail(ctx, SPK_ERR_INVALID_ARG, "row_idx/col_idx/values null");
    return SPK_OK;
}

static spk_status coo_verdict(spk_ctx ctx, const spk_coo *A, int32_t *verdict, int32_t *sorted) {
    *sorted = 1;
    if (A->n_rows < 0 || A->n_cols < 0 || A->nnz < 0) {
        *verdict = SPK_CSR_BAD_SIZE;
        return SPK_OK;
    }
    SPK_HIP(ctx, hipMemsetAsync(ctx->d_flags, 0, sizeof(unsigned), ctx->stream));
    SPK_HIP(ctx, spk::launch_coo_validate(A->n_rows, A->n_cols, A->nnz, A->row_idx, A->col_idx, A->idx_type,
                                          ctx->d_flags, ctx->num_cu * 4, ctx->stream));
    SPK_HIP(ctx, hipMemcpyAsync(ctx->h_flags, ctx->d_flags, sizeof(unsigned), hipMemcpyDeviceToHost, ctx->stream));
    SPK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const unsigned f = *ctx->h_flags;
    *verdict = (f & spk::VFLAG_BAD_FIRST) ? SPK_CSR_BAD_FIRST
                                          : ((f & spk::VFLAG_BAD_COLUMN) ? SPK_CSR_BAD_COLUMN : SPK_CSR_OK);
    *sorted = (f & spk::VFLAG_UNSORTED) ? 0 : 1;
    return SPK_OK;
}

spk_status spk_coo_check(spk_ctx ctx, const spk_coo *A, int32_t *verdict, int32_t *row_sorted) {
    if (!ctx || !verdict || !row_sorted) return SPK_ERR_INVALID_ARG;
    SPK_HIP(ctx, hipSetDevice(ctx->device));
    spk_status s = coo_args(ctx, A);
    if (s != SPK_OK) return s;
    return coo_verdict(ctx, A, verdict, row_sorted);
}

spk_status spk_plan_spmv_coo(spk_ctx ctx, const spk_coo *A, spk_plan *out) {
    if (!ctx || !out) return SPK_ERR_INVALID_ARG;
    *out = nullptr;
    SPK_HIP(ctx, hipSetDevice(ctx->device));
    spk_status s = coo_args(ctx, A);
    if (s != SPK_OK) return s;
    int32_t verdict = 0, sorted = 1;
    if ((s = coo_verdict(ctx, A, &verdict, &sorted)) != SPK_OK) return s;
    if (verdict != SPK_CSR_OK)
        return fail(ctx, SPK_ERR_INVALID_ARG, std::string("malformed COO: ") +
                                                  (verdict == SPK_CSR_BAD_FIRST ? "row index out of range"
                                                                                : verdict_name(verdict)));
    if (!sorted) return fail(ctx, SPK_ERR_INVALID_ARG, "COO entries must be sorted by row");
    spk_csr csr{};
    csr.n_rows = A->n_rows;
    csr.n_cols = A->n_cols;
    csr.nnz = A->nnz;
    csr.ptr_type = A->nnz > INT32_MAX ? SPK_I64 : SPK_I32;
    csr.idx_type = A->idx_type;
    csr.val_type = A->val_type;
    csr.col_idx = A->col_idx;
    csr.values = A->values;
    spk_plan pl = new spk_plan_s();
    pl->ctx = ctx;
    pl->kind = 0;
    const size_t pb = (csr.ptr_type == SPK_I64 ? 8 : 4) * static_cast<size_t>(A->n_rows + 1);
    if (ctx->dpool.get(pb, &pl->coo_rp) != hipSuccess) {
        delete pl;
        return fail(ctx, SPK_ERR_OUT_OF_MEMORY, "COO row pointer");
    }
    csr.row_ptr = pl->coo_rp;
    if (spk::launch_coo_rowptr(A->n_rows, A->nnz, A->row_idx, A->idx_type, pl->coo_rp, csr.ptr_type,
                               ctx->stream) != hipSuccess) {
        (void)hipStreamSynchronize(ctx->stream);
        release_workspace(pl);
        delete pl;
        return fail(ctx, SPK_ERR_DEVICE, "COO row pointer");
    }
    pl->A = to_dev(&csr);
    return finish_spmv_plan(ctx, pl, &csr, out);
}

static spk_status finish_spmv_plan(spk_ctx ctx, spk_plan pl, const spk_csr *A, spk_plan *out) {
    spk_status s = SPK_OK;
    spk_solver_cfg_default(&pl->cfg);
    void *x = nullptr, *y = nullptr;
    const size_t vb = vec_bytes(A->val_type);
    if (A->nnz >= 100000) {
        hipError_t e1 = ctx->dpool.get(std::max<size_t>(1, A->n_cols * vb), &x);
        hipError_t e2 = ctx->dpool.get(std::max<size_t>(1, A->n_rows * vb), &y);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            ctx->dpool.put(x);
            ctx->dpool.put(y);
            release_workspace(pl);
            delete pl;
            return fail(ctx, SPK_ERR_OUT_OF_MEMORY, "tuning buffers");
        }
        (void)hipMemsetAsync(x, 0, A->n_cols * vb, ctx->stream);
    }
    s = build_codes(pl);
    if (s == SPK_OK) s = choose_tune(pl, x, y);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->dpool.put(x);
    ctx->dpool.put(y);
    if (s != SPK_OK) {
        release_workspace(pl);
        delete pl;
        return s;
    }
    pl->info.exec_mode = SPK_EXEC_HOST_LOOP;
    ctx->live_plans++;
    *out = pl;
    return SPK_OK;
}

spk_status spk_plan_solve(spk_ctx ctx, const spk_csr *A, const spk_solver_cfg *cfg_in, spk_plan *out) {
    if (!ctx || !out) return SPK_ERR_INVALID_ARG;
    spk_solver_cfg cfg;
    if (cfg_in) cfg = *cfg_in;
    else spk_solver_cfg_default(&cfg);
    if (cfg.solver != SPK_SOLVER_CG && cfg.solver != SPK_SOLVER_CGS && cfg.solver != SPK_SOLVER_GMRES)
        return fail(ctx, SPK_ERR_INVALID_ARG, "unknown solver");
    if (cfg.solver == SPK_SOLVER_GMRES && (cfg.krylov_dim < 1 || cfg.krylov_dim > spk::kMaxKrylov))
        return fail(ctx, SPK_ERR_INVALID_ARG, "krylov_dim must be in 1..32");
    if (cfg.precond != SPK_PRECOND_NONE && cfg.precond != SPK_PRECOND_JACOBI)
        return fail(ctx, SPK_ERR_INVALID_ARG, "unknown preconditioner");
    if ((cfg.solver == SPK_SOLVER_CGS || cfg.precond == SPK_PRECOND_JACOBI) && cfg.precision != SPK_PREC_FP64)
        return fail(ctx, SPK_ERR_UNSUPPORTED, "CGS and the Jacobi preconditioner run in FP64 precision");
    if (cfg.baseline != SPK_BASELINE_RHS_NORM) return fail(ctx, SPK_ERR_UNSUPPORTED, "only the rhs_norm baseline");
    if (cfg.precision < SPK_PREC_FP64 || cfg.precision > SPK_PREC_MIXED_FP16)
        return fail(ctx, SPK_ERR_INVALID_ARG, "unknown precision");
    if (cfg.max_iters < 0) return fail(ctx, SPK_ERR_INVALID_ARG, "max_iters < 0");
    if (!(cfg.reduction_factor >= 0.0)) return fail(ctx, SPK_ERR_INVALID_ARG, "reduction_factor must be >= 0");
    if (cfg.exec_mode < SPK_EXEC_AUTO || cfg.exec_mode > SPK_EXEC_PERSISTENT)
        return fail(ctx, SPK_ERR_INVALID_ARG, "unknown exec_mode");
    if (cfg.chunk_iters < 0) return fail(ctx, SPK_ERR_INVALID_ARG, "chunk_iters < 0");
    const bool mixed = cfg.precision != SPK_PREC_FP64;
    if (mixed && (!(cfg.inner_reduction > 0.0) || cfg.inner_reduction >= 1.0))
        return fail(ctx, SPK_ERR_INVALID_ARG, "inner_reduction must be in (0, 1)");
    if (mixed && cfg.max_outer < 0) return fail(ctx, SPK_ERR_INVALID_ARG, "max_outer < 0");
    int64_t max_row = 0;
    spk_status s = plan_common(ctx, A, out, &max_row);
    if (s != SPK_OK) return s;
    if (A->n_rows != A->n_cols) return fail(ctx, SPK_ERR_INVALID_ARG, "solve needs a square matrix");
    if (!mixed && A->val_type != SPK_F64) return fail(ctx, SPK_ERR_INVALID_ARG, "FP64 precision needs F64 values");
    if (mixed && A->val_type != SPK_F64 && A->val_type != SPK_F32)
        return fail(ctx, SPK_ERR_INVALID_ARG, "mixed precision needs F64 or F32 values");
    if ((cfg.precision == SPK_PREC_MIXED_BF16 || cfg.precision == SPK_PREC_MIXED_FP16) && A->val_type != SPK_F64)
        return fail(ctx, SPK_ERR_UNSUPPORTED, "BF16 and FP16 inner values are rounded from F64 values only");

    spk_plan pl = new spk_plan_s();
    pl->ctx = ctx;
    pl->kind = 1;
    pl->A = to_dev(A);
    pl->A.max_row = max_row;
    pl->cfg = cfg;
    pl->algo = cfg.solver == SPK_SOLVER_CGS     ? ALGO_CGS
               : cfg.solver == SPK_SOLVER_GMRES ? ALGO_GMRES
               : cfg.precond == SPK_PRECOND_JACOBI ? ALGO_PCG
                                                   : ALGO_CG;
    const int64_t n = A->n_rows;
    const size_t nb = static_cast<size_t>(std::max<int64_t>(n, 1)) * sizeof(double);
    const size_t nf = static_cast<size_t>(std::max<int64_t>(n, 1)) * sizeof(float);
    auto cleanup = [&](spk_status code, const std::string &msg) {
        (void)hipStreamSynchronize(ctx->stream);
        release_workspace(pl);
        delete pl;
        return fail(ctx, code, msg);
    };
    auto dget = [&](size_t bytes, auto **out) {
        void *v = nullptr;
        const bool ok = ctx->dpool.get(bytes, &v) == hipSuccess;
        *out = static_cast<std::remove_reference_t<decltype(*out)>>(v);
        return ok;
    };
    auto hget = [&](size_t bytes, auto **out) {
        void *v = nullptr;
        const bool ok = ctx->hpool.get(bytes, &v) == hipSuccess;
        *out = static_cast<std::remove_reference_t<decltype(*out)>>(v);
        return ok;
    };
    const size_t partial_bytes = sizeof(double) * spk::SITE_COUNT * spk::kSiteWidth * spk::kMaxGrid;
    if (!dget(partial_bytes, &pl->partials)) return cleanup(SPK_ERR_OUT_OF_MEMORY, "partials");
    bool regular = true;   // the pattern decides the loop kind only in the size band between the limits
    if (fused_needs_pattern(cfg, n) && (s = pattern_regular(ctx, pl->A, &regular)) != SPK_OK)
        return cleanup(s, ctx->err);
    s = build_codes(pl);
    if (s != SPK_OK) return cleanup(s, ctx->err);
    const int64_t want = (n + int64_t(spk::kBlock) * 8 - 1) / (int64_t(spk::kBlock) * 8);
    // Streaming kernels: 4 workgroups per CU measured best for HBM copy rates.
    pl->vec_grid = static_cast<int>(std::clamp<int64_t>(want, 1, int64_t(ctx->num_cu) * 4));

    if (!mixed) {
        if (!dget(nb, &pl->r) || !dget(nb, &pl->p) || !dget(nb, &pl->q) || !dget(sizeof(SolveState), &pl->st) ||
            !hget(sizeof(SolveState), &pl->h_st))
            return cleanup(SPK_ERR_OUT_OF_MEMORY, "solve workspace");
        if (cfg.record_history) {
            pl->hist_cap = cfg.max_iters + 1;
            if (!dget(sizeof(double) * pl->hist_cap, &pl->hist)) return cleanup(SPK_ERR_OUT_OF_MEMORY, "history");
        }
        pl->fused = pl->algo == ALGO_CG && fused_loop(cfg, n, regular);
        if (pl->fused && (!dget(nb, &pl->r_b) || !dget(nb, &pl->p_b) || !dget(nb, &pl->q_b)))
            return cleanup(SPK_ERR_OUT_OF_MEMORY, "fused CG workspace");
        if (hipMemsetAsync(pl->st, 0, sizeof(SolveState), ctx->stream) != hipSuccess ||
            hipMemsetAsync(pl->p, 0, nb, ctx->stream) != hipSuccess)
            return cleanup(SPK_ERR_DEVICE, "workspace init");
        std::memset(pl->h_st, 0, sizeof(SolveState));
        if (pl->algo == ALGO_CGS &&
            (!dget(nb, &pl->rt) || !dget(nb, &pl->u) || !dget(nb, &pl->v) || !dget(nb, &pl->uh)))
            return cleanup(SPK_ERR_OUT_OF_MEMORY, "CGS workspace");
        if (pl->algo == ALGO_GMRES) {
            const size_t vbytes =
                sizeof(double) * static_cast<size_t>(spk::gm_ld(std::max<int64_t>(n, 1))) * (cfg.krylov_dim + 1);
            if (!dget(vbytes, &pl->gm_V) || !dget(nb, &pl->gm_w) || !dget(sizeof(spk::GmresState), &pl->gm_st) ||
                !dget(sizeof(double) * (spk::kMaxKrylov + 1) * spk::kMaxGrid, &pl->gm_part))
                return cleanup(SPK_ERR_OUT_OF_MEMORY, "GMRES workspace");
        }
        pl->right_jacobi = (pl->algo == ALGO_CGS || pl->algo == ALGO_GMRES) && cfg.precond == SPK_PRECOND_JACOBI;
        if (pl->right_jacobi) {
            // iterate on A M^{-1}: a scaled copy of the values, once per plan
            pl->A_orig = pl->A;
            if (!dget(nb, &pl->dinv) || !dget(sizeof(unsigned), &pl->diag_flag) ||
                !dget(std::max<size_t>(1, sizeof(double) * A->nnz), &pl->scaled_vals))
                return cleanup(SPK_ERR_OUT_OF_MEMORY, "Jacobi workspace");
            if (hipMemsetAsync(pl->diag_flag, 0, sizeof(unsigned), ctx->stream) != hipSuccess ||
                spk::launch_diag_inv(pl->A, pl->dinv, pl->diag_flag, ctx->stream) != hipSuccess ||
                spk::launch_scale_cols(pl->A, pl->dinv, pl->scaled_vals, ctx->stream) != hipSuccess)
                return cleanup(SPK_ERR_DEVICE, "Jacobi scaling");
            unsigned flag = 0;
            if (hipMemcpyAsync(&flag, pl->diag_flag, sizeof(unsigned), hipMemcpyDeviceToHost, ctx->stream) !=
                    hipSuccess ||
                hipStreamSynchronize(ctx->stream) != hipSuccess)
                return cleanup(SPK_ERR_DEVICE, "Jacobi scaling");
            pl->bad_diag = flag != 0;
            pl->A.va = pl->scaled_vals;
        }
        if (pl->algo == ALGO_PCG) {
            if (!dget(nb, &pl->dinv) || !dget(sizeof(unsigned), &pl->diag_flag))
                return cleanup(SPK_ERR_OUT_OF_MEMORY, "Jacobi workspace");
            if (hipMemsetAsync(pl->diag_flag, 0, sizeof(unsigned), ctx->stream) != hipSuccess ||
                spk::launch_diag_inv(pl->A, pl->dinv, pl->diag_flag, ctx->stream) != hipSuccess)
                return cleanup(SPK_ERR_DEVICE, "Jacobi diagonal");
        }
        if (pl->fused) {
            const spk::FcgBufs<double> f = fcg64(pl);
            if ((s = set_state_x(ctx, pl->st, pl->q)) == SPK_OK) s = choose_tune(pl, pl->p, pl->q, TUNE_FCG, pl->st, &f);
        } else {
            s = choose_tune(pl, pl->p, pl->q, TUNE_CG, pl->st);
        }
        if (s != SPK_OK) return cleanup(s, ctx->err);
    } else {
        if (!dget(nf, &pl->r32) || !dget(nf, &pl->p32) || !dget(nf, &pl->q32) || !dget(nf, &pl->d32) ||
            !dget(sizeof(SolveState), &pl->st_in) || !hget(sizeof(SolveState), &pl->h_st_in) ||
            !dget(4 * sizeof(double), &pl->out_dev) || !hget(4 * sizeof(double), &pl->h_out))
            return cleanup(SPK_ERR_OUT_OF_MEMORY, "mixed workspace");
        // inner matrix view: rounded copy of F64 values, or the F32 values themselves
        pl->A32 = pl->A;
        if (A->val_type == SPK_F64) {
            const int to = cfg.precision == SPK_PREC_MIXED_BF16   ? SPK_BF16
                           : cfg.precision == SPK_PREC_MIXED_FP16 ? SPK_F16
                                                                  : SPK_F32;
            const size_t width = to == SPK_F32 ? 4 : 2;
            void *dst = nullptr;
            if (ctx->dpool.get(std::max<size_t>(1, A->nnz * width), &dst) != hipSuccess)
                return cleanup(SPK_ERR_OUT_OF_MEMORY, "low-precision value copy");
            pl->a32_vals = dst;
            if (A->nnz > 0 && spk::launch_round_values(A->nnz, static_cast<const double *>(A->values), dst, to,
                                                       ctx->num_cu * 4, ctx->stream) != hipSuccess)
                return cleanup(SPK_ERR_DEVICE, "value rounding");
            pl->A32.va = dst;
            pl->A32.val_t = to;
        }
        pl->fused = pl->algo == ALGO_CG && fused_loop(cfg, n, regular);
        if (pl->fused && (!dget(nf, &pl->r32_b) || !dget(nf, &pl->p32_b) || !dget(nf, &pl->q32_b)))
            return cleanup(SPK_ERR_OUT_OF_MEMORY, "fused CG workspace");
        if (pl->algo == ALGO_GMRES) {   // GMRES-IR: FP32 basis
            const size_t vbytes =
                sizeof(float) * static_cast<size_t>(spk::gm_ld(std::max<int64_t>(n, 1))) * (cfg.krylov_dim + 1);
            if (!dget(vbytes, &pl->gm_V) || !dget(nf, &pl->gm_w) || !dget(sizeof(spk::GmresState), &pl->gm_st) ||
                !dget(sizeof(double) * (spk::kMaxKrylov + 1) * spk::kMaxGrid, &pl->gm_part))
                return cleanup(SPK_ERR_OUT_OF_MEMORY, "GMRES workspace");
        }
        if (hipMemsetAsync(pl->st_in, 0, sizeof(SolveState), ctx->stream) != hipSuccess ||
            hipMemsetAsync(pl->p32, 0, nf, ctx->stream) != hipSuccess)
            return cleanup(SPK_ERR_DEVICE, "workspace init");
        std::memset(pl->h_st_in, 0, sizeof(SolveState));
        // Inner SpMV (many launches): timed candidates on A32.  Refinement SpMV
        // (a few launches): launch-shape heuristic on A.
        const CsrDev outer = pl->A;
        pl->A = pl->A32;
        if (pl->fused) {
            const spk::FcgBufs<float> f = fcg32(pl);
            if ((s = set_state_x(ctx, pl->st_in, pl->q32)) == SPK_OK)
                s = choose_tune(pl, pl->p32, pl->q32, TUNE_FCG, pl->st_in, &f);
        } else {
            s = choose_tune(pl, pl->p32, pl->q32, TUNE_CG, pl->st_in);
        }
        pl->A = outer;
        if (s != SPK_OK) return cleanup(s, ctx->err);
        pl->tune32 = pl->tune;
        pl->tune = heuristic_tune(ctx, pl->A);
    }
    int mode = cfg.exec_mode;
    // Automatic choice: the host-issued loop.  On MI355X its launches queue
    // back to back (about 8 us per iteration at the smallest sizes), which
    // measured faster than replaying captured chunks or one cooperative
    // launch with grid barriers.
    if (mode == SPK_EXEC_AUTO) mode = SPK_EXEC_HOST_LOOP;
    if (mode == SPK_EXEC_PERSISTENT && !pl->fused) mode = SPK_EXEC_GRAPH;
    if (pl->algo == ALGO_GMRES) mode = SPK_EXEC_HOST_LOOP;   // cycles read b and x directly
    if (mode == SPK_EXEC_PERSISTENT) {
        // the iterations' matrix and, for a mixed solve, the refinement's
        const CsrDev &Ait = mixed ? pl->A32 : pl->A;
        const int occ = stream_ok(pl->A) && stream_ok(Ait) ? spk::persistent_blocks_per_cu(Ait, mixed ? &pl->A : nullptr)
                                                            : 0;
        const int64_t tiles = std::max<int64_t>((n + spk::kTileRows - 1) / spk::kTileRows, 1);
        // a grid barrier costs about 2 us plus 25-50 ns per workgroup (one
        // agent-scope release and acquire each): at least 8 tiles per
        // workgroup, no fewer than 64 workgroups, at most the resident count
        int64_t g = std::min<int64_t>({std::max<int64_t>(tiles / 8, 64), tiles, int64_t(occ) * ctx->num_cu,
                                       int64_t(spk::kMaxGrid)});
        if (const char *eg = std::getenv("SPK_PERSIST_GRID"))
            if (std::atoi(eg) > 0) g = std::min<int64_t>({int64_t(std::atoi(eg)), int64_t(occ) * ctx->num_cu,
                                                          int64_t(spk::kMaxGrid)});
        void *bv = nullptr, *rv = nullptr;
        if (occ <= 0 || g < 1) {
            mode = SPK_EXEC_GRAPH;
        } else if (ctx->dpool.get(4 * sizeof(unsigned), &bv) != hipSuccess ||
                   (mixed && ctx->dpool.get(sizeof(spk::PersistResult), &rv) != hipSuccess)) {
            if (bv) ctx->dpool.put(bv);
            return cleanup(SPK_ERR_OUT_OF_MEMORY, "barrier words");
        } else {
            pl->bar = static_cast<unsigned *>(bv);
            pl->persist_res = static_cast<spk::PersistResult *>(rv);
            pl->persist_grid = static_cast<int>(g);
            if (hipMemsetAsync(pl->bar, 0, 4 * sizeof(unsigned), ctx->stream) != hipSuccess)
                return cleanup(SPK_ERR_DEVICE, "barrier init");
        }
    }
    pl->info.exec_mode = mode;
    pl->info.chunk_iters = cfg.chunk_iters;
    pl->info.fused_loop = pl->fused ? 1 : 0;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return cleanup(SPK_ERR_DEVICE, "plan sync");
    ctx->live_plans++;
    *out = pl;
    return SPK_OK;
}

spk_status spk_execute_spmv(spk_plan pl, const void *x, void *y) {
    if (!pl || pl->kind != 0) return SPK_ERR_INVALID_ARG;
    spk_ctx ctx = pl->ctx;
    if ((pl->A.n_cols > 0 && !x) || (pl->A.n_rows > 0 && !y)) return fail(ctx, SPK_ERR_INVALID_ARG, "null vector");
    SPK_HIP(ctx, hipSetDevice(ctx->device));
    hipEvent_t e = nullptr;
    spk_status s = prof_begin(pl, &e);
    if (s != SPK_OK) return s;
    SPK_HIP(ctx, spk::launch_spmv(pl->A, pl->tune, x, y, ctx->stream));
    s = prof_end(pl, e);
    if (s != SPK_OK) return s;
    SPK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return prof_collect(pl, pl->ev_used, true);   // this call's launch, if it was timed
}

// Restarted GMRES: each cycle (restart residual, krylov_dim Arnoldi steps,
// triangular solve, x update) is enqueued whole; the state is read once per
// cycle.  Steps after the device ends a cycle return at once.  inner: the
// FP32 solve of a refinement step (A32 d = r32 from d = 0, state st_in, to
// inner_reduction, at most max_iters steps), else the FP64 solve of A x = b.
static spk_status run_gmres(spk_plan pl, const void *b, void *x, bool inner, int64_t max_iters) {
    spk_ctx ctx = pl->ctx;
    const spk_solver_cfg &cfg = pl->cfg;
    const int m = static_cast<int>(cfg.krylov_dim);
    const int64_t n = pl->A.n_rows;
    hipStream_t s = ctx->stream;
    const CsrDev &A = inner ? pl->A32 : pl->A;
    const SpmvTune &tune = inner ? pl->tune32 : pl->tune;
    SolveState *st = inner ? pl->st_in : pl->st;
    SolveState *h_st = inner ? pl->h_st_in : pl->h_st;
    const double tau = inner ? cfg.inner_reduction : cfg.reduction_factor;
    SPK_HIP(ctx, spk::launch_gm_begin(st, pl->gm_st, x, inner ? nullptr : pl->hist, inner ? 0 : pl->hist_cap,
                                      max_iters, s));
    // every cycle but the last completes at least one step
    const int64_t max_cycles = max_iters + 2;
    // profiling: the recorded Arnoldi launches of the current cycle and their
    // step; after the cycle, those past the steps it completed (a cycle that
    // stopped or broke down early) are marked as having done nothing
    std::vector<std::pair<int64_t, int>> recorded;
    int64_t iter_before = 0;
    for (int64_t c = 0; c < max_cycles; ++c) {
        recorded.clear();
        if (inner && c == 0)   // the inner solve starts from d = 0: r = b needs no product
            SPK_HIP(ctx, spk::launch_gm_cycle_start_zero(n, pl->vec_grid, b, pl->gm_V, st, pl->gm_st, pl->partials,
                                                         tau, m, inner, s));
        else
            SPK_HIP(ctx, spk::launch_gm_cycle_start(A, tune, b, x, pl->gm_V, st, pl->gm_st, pl->partials, tau, m,
                                                    inner, s));
        for (int j = 0; j < m; ++j) {
            hipEvent_t e = nullptr;
            int64_t idx = -1;
            spk_status ps = prof_begin(pl, &e, &idx);
            if (ps != SPK_OK) return ps;
            if (idx >= 0) recorded.emplace_back(idx, j);
            SPK_HIP(ctx, spk::launch_gm_step_spmv(A, tune, pl->gm_V, pl->gm_w, j, st, pl->gm_st, inner, s));
            if ((ps = prof_end(pl, e)) != SPK_OK) return ps;
            SPK_HIP(ctx, spk::launch_gm_step_rest(n, pl->vec_grid, pl->gm_V, pl->gm_w, j, m, st, pl->gm_st,
                                                  pl->gm_part, inner, s));
        }
        SPK_HIP(ctx, spk::launch_gm_cycle_end(n, pl->vec_grid, m, pl->gm_V, st, pl->gm_st, inner, s));
        spk_status ps = pull(ctx, h_st, st, sizeof(SolveState));
        if (ps != SPK_OK) return ps;
        const int64_t done = h_st->iter - iter_before;   // steps this cycle completed
        for (const auto &r : recorded)
            if (r.second >= done) pl->ev_ok[static_cast<size_t>(r.first)] = 0;
        iter_before = h_st->iter;
        if (h_st->stop != spk::STOP_RUNNING) return SPK_OK;
    }
    return fail(ctx, SPK_ERR_INTERNAL, "GMRES cycle cap passed without stop");
}

// One cooperative launch for the whole solve (FP64 CG, or the mixed solve
// with its refinement); the barrier gives up after 2 s of waiting.
static spk_status run_persistent(spk_plan pl, const double *b, double *x) {
    spk_ctx ctx = pl->ctx;
    const spk_solver_cfg &cfg = pl->cfg;
    const bool mixed = cfg.precision != SPK_PREC_FP64;
    spk::PersistSolve a{};
    a.b = b;
    a.x = x;
    a.partials = pl->partials;
    a.bar = pl->bar;
    a.spin_ticks = static_cast<uint64_t>(ctx->wall_khz) * 2000ull;
    a.tau = cfg.reduction_factor;
    a.tau_in = cfg.inner_reduction;
    a.max_iters = cfg.max_iters;
    a.max_outer = cfg.max_outer;
    a.remap = pl->tune.xcd_remap;
    a.nt = pl->tune.nt;
    a.true_residual = cfg.true_residual;
    if (mixed) {
        a.f32 = fcg32(pl);
        a.d32 = pl->d32;
        a.res = pl->persist_res;
        a.remap = pl->tune32.xcd_remap;
        a.nt = pl->tune32.nt;
    } else {
        a.f64 = fcg64(pl);
        a.st = pl->st;
        a.hist = pl->hist;
        a.hist_cap = pl->hist_cap;
    }
    SPK_HIP(ctx, hipMemsetAsync(pl->bar, 0, 4 * sizeof(unsigned), ctx->stream));
    SPK_HIP(ctx, spk::launch_persistent(mixed ? pl->A32 : pl->A, mixed ? &pl->A : nullptr, a, pl->persist_grid,
                                        ctx->stream));
    unsigned flags[4] = {0, 0, 0, 0};
    SPK_HIP(ctx, hipMemcpyAsync(flags, pl->bar, sizeof(flags), hipMemcpyDeviceToHost, ctx->stream));
    SPK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (flags[2] != 0) return fail(ctx, SPK_ERR_DEVICE, "persistent solve: a grid barrier timed out");
    return SPK_OK;
}

static spk_status execute_fp64(spk_plan pl, const double *b, double *x, spk_log *L, bool graph) {
    spk_ctx ctx = pl->ctx;
    const spk_solver_cfg &cfg = pl->cfg;
    const int64_t n = pl->A.n_rows;
    spk_status s = SPK_OK;
    if (pl->right_jacobi && pl->bad_diag) {
        // no preconditioner: the initial check reports the breakdown, x unchanged
        SPK_HIP(ctx, spk::launch_pcg_init(pl->A_orig, pl->tune, b, x, pl->dinv, pl->diag_flag, pl->r, pl->p, pl->st,
                                          pl->partials, cfg.reduction_factor, cfg.max_iters, pl->hist, pl->hist_cap,
                                          ctx->stream));
        SPK_HIP(ctx, spk::launch_cg_finalize(pl->A_orig, pl->tune, b, x, pl->st, pl->partials, cfg.true_residual,
                                             ctx->stream));
        if ((s = pull(ctx, pl->h_st, pl->st, sizeof(SolveState))) != SPK_OK) return s;
    } else if (pl->right_jacobi) {
        // solve A M^{-1} u = b for u = M x, then x = M^{-1} u; the residual of
        // the scaled system is the caller's b - A x
        SPK_HIP(ctx, spk::launch_jacobi_vec(n, x, pl->dinv, 1, ctx->stream));
        if (pl->algo == ALGO_GMRES) {
            if ((s = run_gmres(pl, b, x, false, cfg.max_iters)) != SPK_OK) return s;
        } else {
            SPK_HIP(ctx, spk::launch_cg_init(pl->A, pl->tune, b, x, pl->r, pl->rt, pl->st, pl->partials,
                                             cfg.reduction_factor, cfg.max_iters, pl->hist, pl->hist_cap, ctx->stream));
            if ((s = run_loop(pl, LOOP_CGS, cfg.max_iters, graph)) != SPK_OK) return s;
        }
        SPK_HIP(ctx, spk::launch_cg_finalize(pl->A, pl->tune, b, x, pl->st, pl->partials, cfg.true_residual,
                                             ctx->stream));
        SPK_HIP(ctx, spk::launch_jacobi_vec(n, x, pl->dinv, 0, ctx->stream));
        if ((s = pull(ctx, pl->h_st, pl->st, sizeof(SolveState))) != SPK_OK) return s;
    } else if (pl->persist_grid > 0) {
        if ((s = run_persistent(pl, b, x)) != SPK_OK) return s;
        if ((s = pull(ctx, pl->h_st, pl->st, sizeof(SolveState))) != SPK_OK) return s;
    } else if (pl->algo == ALGO_GMRES) {
        if ((s = run_gmres(pl, b, x, false, cfg.max_iters)) != SPK_OK) return s;
        SPK_HIP(ctx, spk::launch_cg_finalize(pl->A, pl->tune, b, x, pl->st, pl->partials, cfg.true_residual,
                                             ctx->stream));
        if ((s = pull(ctx, pl->h_st, pl->st, sizeof(SolveState))) != SPK_OK) return s;
    } else {
        int kind = LOOP_FP64;
        if (pl->algo == ALGO_PCG) {
            SPK_HIP(ctx, spk::launch_pcg_init(pl->A, pl->tune, b, x, pl->dinv, pl->diag_flag, pl->r, pl->p, pl->st,
                                              pl->partials, cfg.reduction_factor, cfg.max_iters, pl->hist,
                                              pl->hist_cap, ctx->stream));
            kind = LOOP_PCG;
        } else {
            if (pl->fused) {
                SPK_HIP(ctx, spk::launch_fcg_init(pl->A, pl->tune, b, x, fcg64(pl), pl->st, pl->partials,
                                                  cfg.reduction_factor, cfg.max_iters, pl->hist, pl->hist_cap,
                                                  ctx->stream));
            } else {
                // CGS: the same initial residual, with the shadow residual rt = r_0 in place of p
                SPK_HIP(ctx, spk::launch_cg_init(pl->A, pl->tune, b, x, pl->r, pl->algo == ALGO_CGS ? pl->rt : pl->p,
                                                 pl->st, pl->partials, cfg.reduction_factor, cfg.max_iters, pl->hist,
                                                 pl->hist_cap, ctx->stream));
            }
            if (pl->algo == ALGO_CGS) kind = LOOP_CGS;
        }
        s = run_loop(pl, kind, cfg.max_iters, graph);
        if (s != SPK_OK) return s;
        SPK_HIP(ctx, spk::launch_cg_finalize(pl->A, pl->tune, b, x, pl->st, pl->partials, cfg.true_residual,
                                             ctx->stream));
        if ((s = pull(ctx, pl->h_st, pl->st, sizeof(SolveState))) != SPK_OK) return s;
    }
    const SolveState &h = *pl->h_st;
    if (pl->profiling) {   // SpMV launches that did work (two per CGS iteration)
        const int64_t per = pl->algo == ALGO_CGS ? 2 : 1;
        // the fused loop: steps 0 .. iterations did work, the next one found
        // the stop; GMRES marks its idle Arnoldi launches itself (every
        // recorded launch is considered)
        const int64_t useful = pl->algo == ALGO_GMRES ? INT64_MAX
                               : pl->fused            ? h.iter + 1
                                                      : per * h.iter + (h.stop == spk::STOP_BREAKDOWN ? 1 : 0);
        if ((s = prof_collect(pl, useful)) != SPK_OK) return s;
    }
    L->iterations = h.iter;
    L->outer_iterations = 0;
    L->implicit_resnorm = h.resnorm;
    L->true_resnorm = cfg.true_residual ? h.true_resnorm : std::nan("");
    L->rhs_norm = h.bnorm;
    L->stop_reason = h.stop;
    return SPK_OK;
}

// Mixed precision with FP64 iterative refinement (Wilkinson/Moler; the
// three-precision form of Carson & Higham 2018 with FP32/BF16 factors):
//   repeat: r = b - A x (FP64); stop if ||r|| <= tau ||b||;
//           solve A32 d = fl32(r) by FP32 CG (FP64 dots) to inner_reduction;
//           x += d.
static spk_status execute_mixed(spk_plan pl, const double *b, double *x, spk_log *L, bool graph) {
    spk_ctx ctx = pl->ctx;
    const spk_solver_cfg &cfg = pl->cfg;
    const int64_t n = pl->A.n_rows;
    if (pl->persist_grid > 0) {
        spk_status s = run_persistent(pl, b, x);
        if (s != SPK_OK) return s;
        spk::PersistResult r{};
        if ((s = pull(ctx, &r, pl->persist_res, sizeof(r))) != SPK_OK) return s;
        L->iterations = r.inner;
        L->outer_iterations = r.outer;
        L->implicit_resnorm = r.rnorm;
        L->true_resnorm = r.rnorm;
        L->rhs_norm = r.bnorm;
        L->stop_reason = r.stop;
        return SPK_OK;
    }
    int64_t inner_total = 0, outer = 0;
    double bnorm = 0.0, rnorm = 0.0;
    int stop = spk::STOP_RUNNING;
    spk_status s = SPK_OK;
    while (true) {
        if (pl->fused)
            SPK_HIP(ctx, spk::launch_fcg_ir_residual(pl->A, pl->tune, b, x, fcg32(pl), pl->d32, pl->st_in,
                                                     pl->partials, cfg.inner_reduction, cfg.max_iters - inner_total,
                                                     pl->out_dev, ctx->stream));
        else
            SPK_HIP(ctx, spk::launch_ir_residual(pl->A, pl->tune, b, x, pl->r32, pl->p32, pl->d32, pl->st_in,
                                                 pl->partials, cfg.inner_reduction, cfg.max_iters - inner_total,
                                                 pl->out_dev, ctx->stream));
        if ((s = pull(ctx, pl->h_out, pl->out_dev, 3 * sizeof(double))) != SPK_OK) return s;
        rnorm = pl->h_out[0];
        bnorm = pl->h_out[2];
        if (!std::isfinite(bnorm) || !std::isfinite(rnorm)) {
            stop = spk::STOP_NON_FINITE;
            break;
        }
        if (bnorm == 0.0) {
            SPK_HIP(ctx, hipMemsetAsync(x, 0, sizeof(double) * n, ctx->stream));
            rnorm = 0.0;
            stop = spk::STOP_CONVERGED;
            break;
        }
        if (rnorm <= cfg.reduction_factor * bnorm) {
            stop = spk::STOP_CONVERGED;
            break;
        }
        if (outer >= cfg.max_outer || inner_total >= cfg.max_iters) {
            stop = spk::STOP_MAX_ITERS;
            break;
        }
        if (pl->algo == ALGO_GMRES) {
            if ((s = run_gmres(pl, pl->r32, pl->d32, true, cfg.max_iters - inner_total)) != SPK_OK) return s;
        } else if ((s = run_loop(pl, LOOP_FP32, cfg.max_iters - inner_total, graph)) != SPK_OK) {
            return s;
        }
        const SolveState &h = *pl->h_st_in;
        inner_total += h.iter;
        if (pl->profiling) {   // this inner solve's SpMV launches that did work
            const int64_t useful = pl->algo == ALGO_GMRES ? INT64_MAX
                                   : pl->fused            ? h.iter + 1
                                                          : h.iter + (h.stop == spk::STOP_BREAKDOWN ? 1 : 0);
            if ((s = prof_collect(pl, useful)) != SPK_OK) return s;
        }
        if ((h.stop == spk::STOP_BREAKDOWN || h.stop == spk::STOP_NON_FINITE) && h.iter == 0) {
            stop = h.stop;
            break;
        }
        SPK_HIP(ctx, spk::launch_ir_correct(n, pl->vec_grid, x, pl->d32, ctx->stream));
        ++outer;
    }
    L->iterations = inner_total;
    L->outer_iterations = outer;
    L->implicit_resnorm = rnorm;
    L->true_resnorm = rnorm;   // the last refinement residual is b - A x in FP64
    L->rhs_norm = bnorm;
    L->stop_reason = stop;
    return SPK_OK;
}

spk_status spk_execute_solve(spk_plan pl, const void *b_in, void *x_in, spk_log *log) {
    if (!pl || pl->kind != 1) return SPK_ERR_INVALID_ARG;
    spk_ctx ctx = pl->ctx;
    const int64_t n = pl->A.n_rows;
    if (n > 0 && (!b_in || !x_in)) return fail(ctx, SPK_ERR_INVALID_ARG, "null vector");
    SPK_HIP(ctx, hipSetDevice(ctx->device));
    spk_log L;
    std::memset(&L, 0, sizeof(L));
    if (n == 0) {
        L.converged = 1;
        L.stop_reason = SPK_STOP_CONVERGED;
        if (log) *log = L;
        return SPK_OK;
    }
    const bool graph = pl->info.exec_mode == SPK_EXEC_GRAPH && !pl->profiling;
    SPK_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    spk_status s = pl->cfg.precision == SPK_PREC_FP64
                       ? execute_fp64(pl, static_cast<const double *>(b_in), static_cast<double *>(x_in), &L, graph)
                       : execute_mixed(pl, static_cast<const double *>(b_in), static_cast<double *>(x_in), &L, graph);
    if (s != SPK_OK) return s;
    SPK_HIP(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    SPK_HIP(ctx, hipEventSynchronize(ctx->ev1));
    float ms = 0.f;
    SPK_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    L.converged = L.stop_reason == SPK_STOP_CONVERGED;
    L.elapsed_ms = ms;
    if (log) *log = L;
    return SPK_OK;
}

// Scratch layout of an allocation-free solve: the solve state, the reduction
// partials, then r, p and q (each 256-byte aligned).
static constexpr size_t kNaPartialBytes = sizeof(double) * spk::SITE_COUNT * spk::kSiteWidth * spk::kMaxGrid;
static constexpr size_t na_align(size_t v) { return (v + 255) & ~size_t(255); }
static constexpr size_t kNaVecBase = na_align(sizeof(SolveState)) + na_align(kNaPartialBytes);

// Rows the scratch holds with v vectors of n doubles (each rounded up to 256 bytes).
static int64_t na_rows(int v) {
    return static_cast<int64_t>((spk::kNoallocScratchBytes - kNaVecBase) / (v * sizeof(double))) - 32;
}

// Vectors of n doubles a solve of n rows keeps in the scratch: r, p, q, and
// their second buffers when it runs the fused loop (as a plan of the same
// configuration and size does).
static int na_vectors(const spk_solver_cfg &cfg, int64_t n) { return fused_loop(cfg, n, true) ? 6 : 3; }

// Whether a solve of n rows fits the scratch.
static bool na_fits(const spk_solver_cfg &cfg, int64_t n) { return n <= na_rows(na_vectors(cfg, n)); }

int64_t spk_noalloc_max_rows(void) {
    // the fused loop (six vectors) runs up to kFusedMaxRows rows, which six
    // vectors hold; above that three vectors (unless the fused loop is forced)
    spk_solver_cfg cfg;
    spk_solver_cfg_default(&cfg);
    return na_fits(cfg, na_rows(3)) ? na_rows(3) : na_rows(6);
}

spk_status spk_solve_noalloc(spk_ctx ctx, const spk_csr *A, const spk_solver_cfg *cfg_in, const void *b_in,
                             void *x_in, spk_log *log) {
    if (!ctx) return SPK_ERR_INVALID_ARG;
    spk_solver_cfg cfg;
    if (cfg_in) cfg = *cfg_in;
    else spk_solver_cfg_default(&cfg);
    if (cfg.solver != SPK_SOLVER_CG || cfg.precond != SPK_PRECOND_NONE || cfg.precision != SPK_PREC_FP64)
        return fail(ctx, SPK_ERR_UNSUPPORTED, "allocation-free solve: FP64 CG without a preconditioner only");
    if (cfg.exec_mode != SPK_EXEC_AUTO && cfg.exec_mode != SPK_EXEC_HOST_LOOP)
        return fail(ctx, SPK_ERR_UNSUPPORTED, "allocation-free solve: host-loop execution only");
    if (cfg.record_history) return fail(ctx, SPK_ERR_UNSUPPORTED, "allocation-free solve keeps no history");
    if (cfg.baseline != SPK_BASELINE_RHS_NORM) return fail(ctx, SPK_ERR_UNSUPPORTED, "only the rhs_norm baseline");
    if (cfg.max_iters < 0) return fail(ctx, SPK_ERR_INVALID_ARG, "max_iters < 0");
    if (!(cfg.reduction_factor >= 0.0)) return fail(ctx, SPK_ERR_INVALID_ARG, "reduction_factor must be >= 0");
    if (cfg.chunk_iters < 0) return fail(ctx, SPK_ERR_INVALID_ARG, "chunk_iters < 0");
    spk_status s = check_csr_args(ctx, A);
    if (s != SPK_OK) return s;
    if (A->n_rows != A->n_cols) return fail(ctx, SPK_ERR_INVALID_ARG, "solve needs a square matrix");
    if (A->val_type != SPK_F64) return fail(ctx, SPK_ERR_INVALID_ARG, "FP64 precision needs F64 values");
    const int64_t n = A->n_rows;
    if (!na_fits(cfg, n))
        return fail(ctx, SPK_ERR_INVALID_ARG,
                    "allocation-free solve: " + std::to_string(n) + " rows exceed the scratch limit of " +
                        std::to_string(na_rows(na_vectors(cfg, n))));
    if (n > 0 && (!b_in || !x_in)) return fail(ctx, SPK_ERR_INVALID_ARG, "null vector");
    if (!ctx->scratch)
        return fail(ctx, SPK_ERR_DEVICE,
                    std::string("allocation-free solve: scratch address lookup failed: ") +
                        hipGetErrorString(ctx->scratch_err));
    SPK_HIP(ctx, hipSetDevice(ctx->device));
    int32_t verdict = 0;
    int64_t max_row = 0;
    if ((s = gpu_verdict(ctx, A, &verdict, &max_row)) != SPK_OK) return s;
    if (verdict != SPK_CSR_OK) return fail(ctx, SPK_ERR_INVALID_ARG, std::string("malformed CSR: ") + verdict_name(verdict));
    spk_log L;
    std::memset(&L, 0, sizeof(L));
    if (n == 0) {
        L.converged = 1;
        L.stop_reason = SPK_STOP_CONVERGED;
        if (log) *log = L;
        return SPK_OK;
    }
    // a plan on the stack whose workspace is the scratch array (its maps and
    // vectors stay empty: no graphs, no profiling events)
    spk_plan_s pl;
    pl.ctx = ctx;
    pl.kind = 1;
    pl.A = to_dev(A);
    pl.A.max_row = max_row;
    pl.cfg = cfg;
    pl.algo = ALGO_CG;
    char *base = static_cast<char *>(ctx->scratch);
    const size_t vb = na_align(sizeof(double) * static_cast<size_t>(n));
    pl.st = reinterpret_cast<SolveState *>(base);
    pl.partials = reinterpret_cast<double *>(base + na_align(sizeof(SolveState)));
    pl.r = reinterpret_cast<double *>(base + kNaVecBase);
    pl.p = reinterpret_cast<double *>(base + kNaVecBase + vb);
    pl.q = reinterpret_cast<double *>(base + kNaVecBase + 2 * vb);
    bool regular = true;
    if (fused_needs_pattern(cfg, n) && (s = pattern_regular(ctx, pl.A, &regular)) != SPK_OK) return s;
    pl.fused = fused_loop(cfg, n, regular);
    if (pl.fused) {
        pl.r_b = reinterpret_cast<double *>(base + kNaVecBase + 3 * vb);
        pl.p_b = reinterpret_cast<double *>(base + kNaVecBase + 4 * vb);
        pl.q_b = reinterpret_cast<double *>(base + kNaVecBase + 5 * vb);
    }
    pl.h_st = ctx->h_noalloc_st;
    std::memset(pl.h_st, 0, sizeof(SolveState));
    const int64_t want = (n + int64_t(spk::kBlock) * 8 - 1) / (int64_t(spk::kBlock) * 8);
    pl.vec_grid = static_cast<int>(std::clamp<int64_t>(want, 1, int64_t(ctx->num_cu) * 4));
    // the launch shape an earlier plan of this shape tuned (read from the
    // context's cache, never added to it), else the heuristic one
    const TuneKey key{pl.A.n_rows, pl.A.n_cols, pl.A.nnz, pl.A.ptr_t, pl.A.idx_t, pl.A.val_t,
                      pl.fused ? TUNE_FCG : TUNE_CG, false,
                      stream_ok(pl.A), pl.A.max_row > spk::kLongRow};
    if (!forced_tune(ctx, pl.A, &pl.tune)) {
        auto hit = ctx->tune_cache.find(key);
        pl.tune = hit != ctx->tune_cache.end() && pl.A.nnz >= 100000 ? hit->second.tune : heuristic_tune(ctx, pl.A);
    }
    pl.info.exec_mode = SPK_EXEC_HOST_LOOP;
    // the scratch keeps the last call's contents: clear the state and p by kernel
    SPK_HIP(ctx, spk::launch_fill_zero(pl.st, na_align(sizeof(SolveState)), ctx->num_cu, ctx->stream));
    SPK_HIP(ctx, spk::launch_fill_zero(pl.p, vb, ctx->num_cu * 4, ctx->stream));
    SPK_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    s = execute_fp64(&pl, static_cast<const double *>(b_in), static_cast<double *>(x_in), &L, false);
    if (s != SPK_OK) {
        (void)hipStreamSynchronize(ctx->stream);
        return s;
    }
    SPK_HIP(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    SPK_HIP(ctx, hipEventSynchronize(ctx->ev1));
    float ms = 0.f;
    SPK_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    L.converged = L.stop_reason == SPK_STOP_CONVERGED;
    L.elapsed_ms = ms;
    if (log) *log = L;
    return SPK_OK;
}

spk_status spk_plan_history(spk_plan pl, double *out, int64_t cap, int64_t *count) {
    if (!pl || !count) return SPK_ERR_INVALID_ARG;
    if (pl->kind != 1 || !pl->hist) return fail(pl->ctx, SPK_ERR_INVALID_ARG, "plan keeps no history");
    const int64_t have = std::min<int64_t>(pl->h_st->iter + 1, pl->hist_cap);
    *count = have;
    const int64_t m = std::min<int64_t>(have, cap);
    if (m > 0 && out) {
        SPK_HIP(pl->ctx, hipSetDevice(pl->ctx->device));
        SPK_HIP(pl->ctx, hipMemcpy(out, pl->hist, sizeof(double) * m, hipMemcpyDeviceToHost));
    }
    return SPK_OK;
}

spk_status spk_plan_get_info(spk_plan pl, spk_plan_info *info) {
    if (!pl || !info) return SPK_ERR_INVALID_ARG;
    *info = pl->info;
    return SPK_OK;
}

spk_status spk_plan_set_profiling(spk_plan pl, int32_t on) {
    if (!pl) return SPK_ERR_INVALID_ARG;
    pl->profiling = on > 0 ? on : 0;
    pl->prof_ms = 0.0;
    pl->prof_count = 0;
    pl->ev_used = 0;
    pl->prof_seq = 0;
    return SPK_OK;
}

spk_status spk_plan_kernel_stats(spk_plan pl, double *total_ms, int64_t *launches) {
    if (!pl || !total_ms || !launches) return SPK_ERR_INVALID_ARG;
    *total_ms = pl->prof_ms;
    *launches = pl->prof_count;
    return SPK_OK;
}

spk_status spk_free(spk_plan pl) {
    if (!pl) return SPK_OK;
    spk_ctx ctx = pl->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &g : pl->graphs) (void)hipGraphExecDestroy(g.second);
    for (auto &e : pl->ev_pool) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    release_workspace(pl);
    ctx->live_plans--;
    delete pl;
    return SPK_OK;
}

spk_status spk_gather_probe(spk_ctx ctx, const double *src, int64_t n_src, const int32_t *idx, int64_t m,
                            double *dst, double *ms) {
    if (!ctx) return SPK_ERR_INVALID_ARG;
    if (n_src < 1 || m < 0 || n_src > INT32_MAX || !src || (m > 0 && (!idx || !dst)))
        return fail(ctx, SPK_ERR_INVALID_ARG, "gather probe: bad sizes or null pointers");
    SPK_HIP(ctx, hipSetDevice(ctx->device));
    // the indices must stay in range: checked on the GPU first (the CSR
    // validation kernel on a one-row matrix whose columns are idx)
    spk_csr probe{};
    probe.n_rows = 1;
    probe.n_cols = n_src;
    probe.nnz = m;
    probe.ptr_type = SPK_I64;
    probe.idx_type = SPK_I32;
    probe.val_type = SPK_F64;
    int64_t rp_h[2] = {0, m};
    void *rp_d = nullptr;
    if (ctx->dpool.get(sizeof(rp_h), &rp_d) != hipSuccess) return fail(ctx, SPK_ERR_OUT_OF_MEMORY, "gather probe");
    probe.row_ptr = rp_d;
    probe.col_idx = idx;
    probe.values = dst;
    int32_t verdict = 0;
    spk_status s = SPK_OK;
    if (hipMemcpyAsync(rp_d, rp_h, sizeof(rp_h), hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
        s = fail(ctx, SPK_ERR_DEVICE, "gather probe: upload");
    if (s == SPK_OK) s = gpu_verdict(ctx, &probe, &verdict);
    ctx->dpool.put(rp_d);
    if (s != SPK_OK) return s;
    if (verdict != SPK_CSR_OK) return fail(ctx, SPK_ERR_INVALID_ARG, "gather probe: an index is out of range");
    const int grid = std::min(ctx->num_cu * 8, spk::kMaxGrid);
    SPK_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    if (m > 0) SPK_HIP(ctx, spk::launch_gather(src, idx, dst, m, grid, ctx->stream));
    SPK_HIP(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    SPK_HIP(ctx, hipEventSynchronize(ctx->ev1));
    float t = 0.f;
    SPK_HIP(ctx, hipEventElapsedTime(&t, ctx->ev0, ctx->ev1));
    if (ms) *ms = t;
    return SPK_OK;
}

spk_status spk_stream_copy(spk_ctx ctx, const void *src, void *dst, size_t bytes, double *ms) {
    if (!ctx || !src || !dst || (bytes % 16) != 0 || (reinterpret_cast<uintptr_t>(src) & 15) ||
        (reinterpret_cast<uintptr_t>(dst) & 15))
        return fail(ctx, SPK_ERR_INVALID_ARG, "copy needs 16-byte aligned pointers and size");
    SPK_HIP(ctx, hipSetDevice(ctx->device));
    const int grid = std::min(ctx->num_cu * 4, spk::kMaxGrid);
    SPK_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    SPK_HIP(ctx, spk::launch_copy(src, dst, bytes, grid, ctx->stream));
    SPK_HIP(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    SPK_HIP(ctx, hipEventSynchronize(ctx->ev1));
    float t = 0.f;
    SPK_HIP(ctx, hipEventElapsedTime(&t, ctx->ev0, ctx->ev1));
    if (ms) *ms = t;
    return SPK_OK;
}

}  // extern "C"
