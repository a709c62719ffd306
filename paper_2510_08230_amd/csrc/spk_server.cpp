// Continuous-batching solve server (spk_server_* in include/spk.h).
//
// Requests (CSR matrix, b, x on the device) arrive from any host thread.  A
// worker thread owns the GPU side: it validates each request, admits it into
// a free slot when its workspace fits the HBM budget, rebuilds the device
// tile/slot tables, replays a captured graph of K batched ticks, reads every
// live slot's status once per K ticks, and retires finished requests (their
// slot and workspace become free for queued ones).  Requests that arrive
// while others run are admitted between tick batches, so their work overlaps
// on the device with the requests already in flight.
#include "spk.h"
#include "spk_internal.h"
#include "spk_launch.h"
#include "spk_pool.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int64_t tiles_of(int64_t n) { return (n + spk::kTileRows - 1) / spk::kTileRows; }

size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// Workspace one request needs: r, p, q, d (n each; FP32 for a mixed
// request, FP64 for an FP64 one), the FP32 value copy (nnz; mixed only), the
// per-tile partial sums, and 32-bit copies of 64-bit row pointers (n + 1)
// and columns (nnz): the tick kernels read 32-bit indices.
size_t request_bytes(int64_t n, int64_t nnz, bool fp64, bool ptr64 = false, bool idx64 = false) {
    const size_t es = fp64 ? sizeof(double) : sizeof(float);
    const size_t vec = align256(es * static_cast<size_t>(std::max<int64_t>(n, 1)));
    const size_t copy = fp64 ? 0 : align256(sizeof(float) * static_cast<size_t>(std::max<int64_t>(nnz, 1)));
    const size_t rp32 = ptr64 ? align256(sizeof(int32_t) * static_cast<size_t>(n + 1)) : 0;
    const size_t ci32 = idx64 ? align256(sizeof(int32_t) * static_cast<size_t>(std::max<int64_t>(nnz, 1))) : 0;
    return 4 * vec + copy + rp32 + ci32 +
           align256(sizeof(double) * spk::kPartSites * static_cast<size_t>(std::max<int64_t>(tiles_of(n), 1)));
}

struct Request {
    uint64_t ticket = 0;
    spk_csr A{};
    const double *b = nullptr;
    double *x = nullptr;
    int64_t submit_ns = 0;
    double tau = 0.0, tau_in = 0.0;   // this request's stop tests
    int64_t max_iters = 0, max_outer = 0;
    bool fp64 = false;                 // SPK_PREC_FP64 (else SPK_PREC_MIXED_FP32)
    bool ptr64 = false, idx64 = false; // 64-bit row pointers / columns (narrowed at admission)
};

// The LDS tiles stage a tile's values and columns with 16-byte DMA loads,
// which need 16-byte aligned arrays; other requests read them directly.
bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Configuration checks shared by create (server default) and submit (per request).
bool cfg_supported(const spk_solver_cfg &c) {
    return c.solver == SPK_SOLVER_CG && c.precond == SPK_PRECOND_NONE &&
           (c.precision == SPK_PREC_MIXED_FP32 || c.precision == SPK_PREC_FP64);
}
bool cfg_valid(const spk_solver_cfg &c) {
    return c.reduction_factor >= 0.0 && c.inner_reduction > 0.0 && c.inner_reduction < 1.0 && c.max_iters >= 0 &&
           c.max_outer >= 0;
}

struct Result {
    int32_t done = 0;
    spk_status status = SPK_OK;
    spk_log log{};
    int64_t submit_ns = 0, admit_ns = 0, done_ns = 0;
};

struct Slot {
    bool live = false;
    Request req;
    void *ws = nullptr;
    size_t bytes = 0;
    int64_t tiles = 0;
    int64_t admit_ns = 0;
};

}  // namespace

struct spk_server_s {
    int device = 0;
    int num_cu = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0;
    int max_slots = 0;
    spk_solver_cfg cfg{};
    spk::DevicePool pool;
    // device tables (fixed pointers: the captured tick graph refers to them)
    int32_t *d_counts = nullptr;
    int2 *d_tiles = nullptr;
    int32_t *d_slots = nullptr;
    spk::SlotDesc *d_desc = nullptr;
    spk::SlotState *d_state = nullptr;
    spk::SlotStatus *d_status = nullptr;
    unsigned *d_flags = nullptr;
    // pinned staging
    int32_t *h_counts = nullptr;
    int2 *h_tiles = nullptr;
    int32_t *h_slots = nullptr;
    spk::SlotDesc *h_desc = nullptr;
    spk::SlotState *h_state = nullptr;
    spk::SlotStatus *h_status = nullptr;
    unsigned *h_flags = nullptr;
    int64_t cap_tiles = 0;
    spk::BatchDev B{};
    hipGraphExec_t tick_graph = nullptr;
    int ticks_per_poll = 4;
    // host state (worker thread only)
    std::vector<Slot> slots;
    std::deque<Request> waiting;
    size_t bytes_in_use = 0;
    int64_t live_tiles = 0;
    // shared with submitters
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<Request> incoming;
    std::unordered_map<uint64_t, Result> results;
    uint64_t next_ticket = 1;
    int64_t outstanding = 0;
    bool stopping = false;
    std::string err;
    spk_server_stats stats{};
    std::thread worker;
};

namespace {

void finish(spk_server srv, const Request &r, spk_status status, const spk_log &log, int64_t admit_ns) {
    std::lock_guard<std::mutex> lk(srv->mu);
    Result &res = srv->results[r.ticket];
    res.done = 1;
    res.status = status;
    res.log = log;
    res.admit_ns = admit_ns;
    res.done_ns = now_ns();
    srv->outstanding -= 1;
    if (status == SPK_OK) srv->stats.completed += 1;
    else srv->stats.failed += 1;
    srv->cv_done.notify_all();
}

bool hip_ok(spk_server srv, hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->err = std::string(what) + ": " + hipGetErrorString(e);
    return false;
}

// GPU well-formedness check of a request's CSR (same kernel as the plans use).
bool request_valid(spk_server srv, const Request &r) {
    spk::CsrDev d{r.A.n_rows, r.A.n_cols, r.A.nnz, r.A.ptr_type, r.A.idx_type, r.A.val_type,
                  r.A.row_ptr, r.A.col_idx, r.A.values};
    if (!hip_ok(srv, hipMemsetAsync(srv->d_flags, 0, 2 * sizeof(unsigned), srv->stream), "flags")) return false;
    if (!hip_ok(srv, spk::launch_validate(d, srv->d_flags, srv->num_cu * 4, srv->stream), "validate")) return false;
    if (!hip_ok(srv, hipMemcpyAsync(srv->h_flags, srv->d_flags, sizeof(unsigned), hipMemcpyDeviceToHost, srv->stream),
                "flags copy"))
        return false;
    if (!hip_ok(srv, hipStreamSynchronize(srv->stream), "validate sync")) return false;
    return *srv->h_flags == 0;
}

// Admit waiting requests in arrival order while a slot is free and the
// request's workspace fits the remaining budget and tile capacity.
bool admit(spk_server srv) {
    bool changed = false;
    while (!srv->waiting.empty()) {
        Request &r = srv->waiting.front();
        const int64_t n = r.A.n_rows;
        const size_t bytes = request_bytes(n, r.A.nnz, r.fp64, r.ptr64, r.idx64);
        const int64_t t = tiles_of(n);
        int free_slot = -1;
        for (int i = 0; i < srv->max_slots; ++i)
            if (!srv->slots[i].live) {
                free_slot = i;
                break;
            }
        if (free_slot < 0 || srv->bytes_in_use + bytes > srv->budget || srv->live_tiles + t > srv->cap_tiles) break;
        Request req = r;
        srv->waiting.pop_front();
        spk_log empty{};
        if (!request_valid(srv, req)) {
            finish(srv, req, SPK_ERR_INVALID_ARG, empty, 0);
            continue;
        }
        void *ws = nullptr;
        if (srv->pool.get(bytes, &ws) != hipSuccess) {   // budget is above free memory: retry later
            srv->waiting.push_front(req);
            break;
        }
        char *cur = static_cast<char *>(ws);
        auto carve = [&](size_t b) {
            char *p = cur;
            cur += align256(b);
            return p;
        };
        const size_t nn = static_cast<size_t>(std::max<int64_t>(n, 1));
        spk::SlotDesc &D = srv->h_desc[free_slot];
        std::memset(&D, 0, sizeof(D));
        D.n = n;
        D.nnz = req.A.nnz;
        D.tiles = t;
        D.rp = static_cast<const int32_t *>(req.A.row_ptr);
        D.ci = static_cast<const int32_t *>(req.A.col_idx);
        int32_t *rp32 = nullptr, *ci32 = nullptr;
        D.va64 = static_cast<const double *>(req.A.values);
        D.fp64 = req.fp64 ? 1 : 0;
        float *va32 = nullptr;
        if (req.fp64) {
            D.r64 = reinterpret_cast<double *>(carve(sizeof(double) * nn));
            D.p64 = reinterpret_cast<double *>(carve(sizeof(double) * nn));
            D.q64 = reinterpret_cast<double *>(carve(sizeof(double) * nn));
            D.d64 = reinterpret_cast<double *>(carve(sizeof(double) * nn));
        } else {
            D.r = reinterpret_cast<float *>(carve(sizeof(float) * nn));
            D.p = reinterpret_cast<float *>(carve(sizeof(float) * nn));
            D.q = reinterpret_cast<float *>(carve(sizeof(float) * nn));
            D.d = reinterpret_cast<float *>(carve(sizeof(float) * nn));
            va32 = reinterpret_cast<float *>(carve(sizeof(float) * static_cast<size_t>(std::max<int64_t>(req.A.nnz, 1))));
        }
        D.va32 = va32;
        if (req.ptr64) D.rp = rp32 = reinterpret_cast<int32_t *>(carve(sizeof(int32_t) * static_cast<size_t>(n + 1)));
        if (req.idx64)
            D.ci = ci32 = reinterpret_cast<int32_t *>(
                carve(sizeof(int32_t) * static_cast<size_t>(std::max<int64_t>(req.A.nnz, 1))));
        D.part = reinterpret_cast<double *>(carve(sizeof(double) * spk::kPartSites * static_cast<size_t>(std::max<int64_t>(t, 1))));
        D.b = req.b;
        D.x = req.x;
        D.tau = req.tau;
        D.tau_in = req.tau_in;
        D.max_iters = req.max_iters;
        D.max_outer = req.max_outer;
        // the slot's FP32 values are carved 256-byte aligned; the caller's
        // FP64 values and columns decide whether tiles are DMA-staged
        D.stage = (aligned16(D.ci) && aligned16(D.va64)) ? 1 : 0;
        spk::SlotState &S = srv->h_state[free_slot];
        std::memset(&S, 0, sizeof(S));
        S.phase = spk::PH_OUTER;
        S.next_phase = spk::PH_OUTER;
        bool ok = true;
        if (rp32)
            ok = hip_ok(srv, spk::launch_narrow_i32(n + 1, static_cast<const int64_t *>(req.A.row_ptr), rp32,
                                                    srv->num_cu * 4, srv->stream), "row pointers");
        if (ok && ci32)
            ok = hip_ok(srv, spk::launch_narrow_i32(req.A.nnz, static_cast<const int64_t *>(req.A.col_idx), ci32,
                                                    srv->num_cu * 4, srv->stream), "columns");
        if (ok && req.A.nnz > 0 && !req.fp64)
            ok = hip_ok(srv, spk::launch_round_f32(req.A.nnz, D.va64, va32, srv->num_cu * 4, srv->stream), "round");
        ok = ok && hip_ok(srv, hipMemcpyAsync(srv->d_desc + free_slot, &D, sizeof(D), hipMemcpyHostToDevice, srv->stream),
                          "desc upload");
        ok = ok && hip_ok(srv, hipMemcpyAsync(srv->d_state + free_slot, &S, sizeof(S), hipMemcpyHostToDevice, srv->stream),
                          "state upload");
        if (!ok) {
            srv->pool.put(ws);
            finish(srv, req, SPK_ERR_DEVICE, empty, 0);
            continue;
        }
        Slot &sl = srv->slots[free_slot];
        sl.live = true;
        sl.req = req;
        sl.ws = ws;
        sl.bytes = bytes;
        sl.tiles = t;
        sl.admit_ns = now_ns();
        srv->bytes_in_use += bytes;
        srv->live_tiles += t;
        changed = true;
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stats.admitted += 1;
        srv->stats.peak_bytes = std::max<int64_t>(srv->stats.peak_bytes, static_cast<int64_t>(srv->bytes_in_use));
        srv->stats.peak_device_bytes = std::max<int64_t>(
            srv->stats.peak_device_bytes, static_cast<int64_t>(srv->pool.in_use() + srv->pool.cached()));
    }
    return changed;
}

bool rebuild_tables(spk_server srv) {
    // the staging arrays may still feed a previous upload: let it finish first
    if (!hip_ok(srv, hipStreamSynchronize(srv->stream), "table sync")) return false;
    int32_t nt = 0, ns = 0;
    for (int i = 0; i < srv->max_slots; ++i) {
        const Slot &sl = srv->slots[i];
        if (!sl.live) continue;
        srv->h_slots[ns++] = i;
        for (int64_t t = 0; t < sl.tiles; ++t) srv->h_tiles[nt++] = make_int2(i, static_cast<int>(t));
    }
    srv->h_counts[0] = nt;
    srv->h_counts[1] = ns;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stats.peak_slots = std::max<int64_t>(srv->stats.peak_slots, ns);
    }
    bool ok = hip_ok(srv, hipMemcpyAsync(srv->d_counts, srv->h_counts, 2 * sizeof(int32_t), hipMemcpyHostToDevice,
                                         srv->stream), "counts upload");
    if (nt > 0)
        ok = ok && hip_ok(srv, hipMemcpyAsync(srv->d_tiles, srv->h_tiles, sizeof(int2) * nt, hipMemcpyHostToDevice,
                                              srv->stream), "tiles upload");
    if (ns > 0)
        ok = ok && hip_ok(srv, hipMemcpyAsync(srv->d_slots, srv->h_slots, sizeof(int32_t) * ns, hipMemcpyHostToDevice,
                                              srv->stream), "slots upload");
    return ok;
}

bool run_ticks(spk_server srv) {
    if (!srv->tick_graph) {
        hipStream_t cap = nullptr;
        if (!hip_ok(srv, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "capture stream")) return false;
        hipGraph_t g = nullptr;
        bool ok = hip_ok(srv, hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
        for (int k = 0; ok && k < srv->ticks_per_poll; ++k) ok = hip_ok(srv, spk::launch_batch_tick(srv->B, cap), "tick");
        hipError_t e = hipStreamEndCapture(cap, &g);
        ok = ok && hip_ok(srv, e, "end capture");
        if (ok) ok = hip_ok(srv, hipGraphInstantiate(&srv->tick_graph, g, nullptr, nullptr, 0), "instantiate");
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(cap);
        if (!ok) return false;
    }
    if (!hip_ok(srv, hipGraphLaunch(srv->tick_graph, srv->stream), "graph launch")) return false;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stats.ticks += srv->ticks_per_poll;
    return true;
}

// Read every live slot's status; retire the finished ones.
bool retire(spk_server srv, bool *changed) {
    *changed = false;
    if (!hip_ok(srv, hipMemcpyAsync(srv->h_status, srv->d_status, sizeof(spk::SlotStatus) * srv->max_slots,
                                    hipMemcpyDeviceToHost, srv->stream), "status copy"))
        return false;
    if (!hip_ok(srv, hipStreamSynchronize(srv->stream), "tick sync")) return false;
    for (int i = 0; i < srv->max_slots; ++i) {
        Slot &sl = srv->slots[i];
        if (!sl.live) continue;
        const spk::SlotStatus &st = srv->h_status[i];
        if (st.phase != spk::PH_DONE) continue;
        spk_log log{};
        log.iterations = st.iters;
        log.outer_iterations = st.outer;
        log.implicit_resnorm = st.rnorm;
        log.true_resnorm = st.rnorm;
        log.rhs_norm = st.bnorm;
        log.stop_reason = st.stop;
        log.converged = st.stop == SPK_STOP_CONVERGED;
        finish(srv, sl.req, SPK_OK, log, sl.admit_ns);
        srv->pool.put(sl.ws);
        srv->bytes_in_use -= sl.bytes;
        srv->live_tiles -= sl.tiles;
        sl = Slot{};
        srv->h_status[i].phase = spk::PH_FREE;
        *changed = true;
    }
    return true;
}

void fail_all(spk_server srv) {
    spk_log empty{};
    for (Slot &sl : srv->slots)
        if (sl.live) {
            finish(srv, sl.req, SPK_ERR_DEVICE, empty, sl.admit_ns);
            sl = Slot{};
        }
    for (const Request &r : srv->waiting) finish(srv, r, SPK_ERR_DEVICE, empty, 0);
    srv->waiting.clear();
}

void worker_main(spk_server srv) {
    if (hipSetDevice(srv->device) != hipSuccess) return;
    bool broken = false;
    while (true) {
        int live = 0;
        for (const Slot &sl : srv->slots) live += sl.live ? 1 : 0;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->cv.wait(lk, [&] { return srv->stopping || !srv->incoming.empty() || live > 0 || !srv->waiting.empty(); });
            while (!srv->incoming.empty()) {
                srv->waiting.push_back(srv->incoming.front());
                srv->incoming.pop_front();
            }
            if (srv->stopping && srv->waiting.empty() && live == 0) break;
        }
        if (broken) {
            fail_all(srv);
            continue;
        }
        bool changed = admit(srv);
        live = 0;
        for (const Slot &sl : srv->slots) live += sl.live ? 1 : 0;
        if (live == 0) {
            if (!srv->waiting.empty()) {   // nothing runs and the head cannot be admitted: over budget
                spk_log empty{};
                finish(srv, srv->waiting.front(), SPK_ERR_BUDGET, empty, 0);
                srv->waiting.pop_front();
            }
            continue;
        }
        if (changed && !rebuild_tables(srv)) broken = true;
        if (!broken && !run_ticks(srv)) broken = true;
        bool retired = false;
        if (!broken && !retire(srv, &retired)) broken = true;
        if (!broken && retired && !rebuild_tables(srv)) broken = true;
    }
}

}  // namespace

extern "C" {

size_t spk_server_request_bytes(int64_t n, int64_t nnz) { return request_bytes(n, nnz, false); }

size_t spk_server_request_bytes_prec(int32_t precision, int64_t n, int64_t nnz) {
    if (precision == SPK_PREC_FP64) return request_bytes(n, nnz, true);
    if (precision == SPK_PREC_MIXED_FP32) return request_bytes(n, nnz, false);
    return 0;
}

size_t spk_server_request_bytes_csr(const spk_csr *A, int32_t precision) {
    if (!A || A->n_rows < 0 || A->nnz < 0) return 0;
    if ((A->ptr_type != SPK_I32 && A->ptr_type != SPK_I64) || (A->idx_type != SPK_I32 && A->idx_type != SPK_I64))
        return 0;
    if (precision != SPK_PREC_FP64 && precision != SPK_PREC_MIXED_FP32) return 0;
    return request_bytes(A->n_rows, A->nnz, precision == SPK_PREC_FP64, A->ptr_type == SPK_I64,
                         A->idx_type == SPK_I64);
}

spk_status spk_server_create(spk_ctx ctx, size_t hbm_budget_bytes, int32_t max_slots, const spk_solver_cfg *cfg,
                             spk_server *out) {
    if (!ctx || !out || max_slots < 1 || max_slots > 65536 || hbm_budget_bytes == 0) return SPK_ERR_INVALID_ARG;
    *out = nullptr;
    spk_solver_cfg c;
    if (cfg) c = *cfg;
    else spk_solver_cfg_default(&c);
    if (!cfg_supported(c)) return SPK_ERR_UNSUPPORTED;
    if (!cfg_valid(c)) return SPK_ERR_INVALID_ARG;
    const int dev = spk::ctx_device(ctx);
    if (hipSetDevice(dev) != hipSuccess) return SPK_ERR_DEVICE;
    spk_server srv = new spk_server_s();
    srv->device = dev;
    srv->budget = hbm_budget_bytes;
    srv->max_slots = max_slots;
    srv->cfg = c;
    // the budget bounds the device memory the request pool holds, cached
    // blocks included (exact-size reuse, so a request's charge is its block)
    srv->pool.set_budget_mode(true);
    srv->pool.set_cap(hbm_budget_bytes);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete srv;
        return SPK_ERR_DEVICE;
    }
    srv->num_cu = prop.multiProcessorCount;
    srv->cap_tiles = std::min<int64_t>(static_cast<int64_t>(hbm_budget_bytes / 4096) + 1, int64_t(1) << 21);
    srv->slots.resize(max_slots);
    const size_t ms = static_cast<size_t>(max_slots);
    bool ok = hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc(&srv->d_counts, 2 * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&srv->d_tiles, sizeof(int2) * srv->cap_tiles) == hipSuccess &&
              hipMalloc(&srv->d_slots, sizeof(int32_t) * ms) == hipSuccess &&
              hipMalloc(&srv->d_desc, sizeof(spk::SlotDesc) * ms) == hipSuccess &&
              hipMalloc(&srv->d_state, sizeof(spk::SlotState) * ms) == hipSuccess &&
              hipMalloc(&srv->d_status, sizeof(spk::SlotStatus) * ms) == hipSuccess &&
              hipMalloc(&srv->d_flags, 2 * sizeof(unsigned)) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void **>(&srv->h_counts), 2 * sizeof(int32_t), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void **>(&srv->h_tiles), sizeof(int2) * srv->cap_tiles, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void **>(&srv->h_slots), sizeof(int32_t) * ms, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void **>(&srv->h_desc), sizeof(spk::SlotDesc) * ms, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void **>(&srv->h_state), sizeof(spk::SlotState) * ms, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void **>(&srv->h_status), sizeof(spk::SlotStatus) * ms, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void **>(&srv->h_flags), 2 * sizeof(unsigned), hipHostMallocDefault) == hipSuccess;
    if (ok) {
        std::memset(srv->h_status, 0, sizeof(spk::SlotStatus) * ms);
        srv->h_counts[0] = srv->h_counts[1] = 0;
        ok = hipMemsetAsync(srv->d_state, 0, sizeof(spk::SlotState) * ms, srv->stream) == hipSuccess &&
             hipMemsetAsync(srv->d_status, 0, sizeof(spk::SlotStatus) * ms, srv->stream) == hipSuccess &&
             hipMemsetAsync(srv->d_counts, 0, 2 * sizeof(int32_t), srv->stream) == hipSuccess &&
             hipStreamSynchronize(srv->stream) == hipSuccess;
    }
    if (!ok) {
        spk_server_destroy(srv);
        return SPK_ERR_OUT_OF_MEMORY;
    }
    const int occ = spk::batch_tile_blocks_per_cu();
    // tile launches: each XCD walks a contiguous eighth of the tick's tile
    // list (which is ordered request by request), so a request's gathered
    // vector is read into few L2s; the matrix streams non-temporally.
    // SPK_BATCH_TILES="remap=R,nt=T" overrides either.
    int remap = 1, nt = 1;
    if (const char *e = std::getenv("SPK_BATCH_TILES")) {
        if (const char *r = std::strstr(e, "remap=")) remap = std::atoi(r + 6);
        if (const char *t = std::strstr(e, "nt=")) nt = std::atoi(t + 3);
    }
    srv->B = spk::BatchDev{srv->d_counts, srv->d_tiles, srv->d_slots, srv->d_desc, srv->d_state, srv->d_status,
                           std::min(srv->num_cu * occ, spk::kMaxGrid), std::min(srv->num_cu * 4, max_slots),
                           remap, nt};
    srv->stats.budget_bytes = static_cast<int64_t>(hbm_budget_bytes);
    srv->stats.max_slots = max_slots;
    srv->worker = std::thread(worker_main, srv);
    *out = srv;
    return SPK_OK;
}

spk_status spk_server_submit(spk_server srv, const spk_csr *A, const void *b, void *x, uint64_t *ticket) {
    return spk_server_submit_cfg(srv, A, b, x, nullptr, ticket);
}

spk_status spk_server_submit_cfg(spk_server srv, const spk_csr *A, const void *b, void *x, const spk_solver_cfg *cfg,
                                 uint64_t *ticket) {
    if (!srv || !A || !ticket) return SPK_ERR_INVALID_ARG;
    const spk_solver_cfg &c = cfg ? *cfg : srv->cfg;
    if (cfg && !cfg_supported(c)) return SPK_ERR_UNSUPPORTED;
    if (cfg && !cfg_valid(c)) return SPK_ERR_INVALID_ARG;
    if (A->n_rows != A->n_cols || A->n_rows < 1 || A->nnz < 0) return SPK_ERR_INVALID_ARG;
    if ((A->ptr_type != SPK_I32 && A->ptr_type != SPK_I64) || (A->idx_type != SPK_I32 && A->idx_type != SPK_I64) ||
        A->val_type != SPK_F64)
        return SPK_ERR_UNSUPPORTED;
    // the tick kernels read 32-bit indices: 64-bit ones are narrowed, so
    // their values (at most n and nnz) must fit
    if ((A->ptr_type == SPK_I64 || A->idx_type == SPK_I64) && (A->n_rows >= INT32_MAX || A->nnz >= INT32_MAX))
        return SPK_ERR_UNSUPPORTED;
    if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->values)) || !b || !x) return SPK_ERR_INVALID_ARG;
    const bool fp64 = c.precision == SPK_PREC_FP64;
    const bool ptr64 = A->ptr_type == SPK_I64, idx64 = A->idx_type == SPK_I64;
    if (request_bytes(A->n_rows, A->nnz, fp64, ptr64, idx64) > srv->budget || tiles_of(A->n_rows) > srv->cap_tiles)
        return SPK_ERR_BUDGET;
    if (tiles_of(A->n_rows) > INT32_MAX) return SPK_ERR_UNSUPPORTED;
    Request r;
    r.A = *A;
    r.b = static_cast<const double *>(b);
    r.x = static_cast<double *>(x);
    r.submit_ns = now_ns();
    r.tau = c.reduction_factor;
    r.tau_in = c.inner_reduction;
    r.max_iters = c.max_iters;
    r.max_outer = c.max_outer;
    r.fp64 = fp64;
    r.ptr64 = ptr64;
    r.idx64 = idx64;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stopping) return SPK_ERR_INVALID_ARG;
        r.ticket = srv->next_ticket++;
        Result &res = srv->results[r.ticket];
        res.submit_ns = r.submit_ns;
        srv->outstanding += 1;
        srv->stats.submitted += 1;
        srv->incoming.push_back(r);
    }
    srv->cv.notify_one();
    *ticket = r.ticket;
    return SPK_OK;
}

spk_status spk_server_poll(spk_server srv, uint64_t ticket, int32_t *done, spk_log *log, int64_t *latency_ns) {
    if (!srv || !done) return SPK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->results.find(ticket);
    if (it == srv->results.end()) return SPK_ERR_INVALID_ARG;
    *done = it->second.done;
    if (!it->second.done) return SPK_OK;
    if (log) *log = it->second.log;
    if (latency_ns) *latency_ns = it->second.done_ns - it->second.submit_ns;
    return it->second.status;
}

spk_status spk_server_drain(spk_server srv) {
    if (!srv) return SPK_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->outstanding == 0; });
    return srv->err.empty() ? SPK_OK : SPK_ERR_DEVICE;
}

spk_status spk_server_get_stats(spk_server srv, spk_server_stats *st) {
    if (!srv || !st) return SPK_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    *st = srv->stats;
    return SPK_OK;
}

const char *spk_server_last_error(spk_server srv) {
    if (!srv) return "null server";
    std::lock_guard<std::mutex> lk(srv->mu);
    return srv->err.c_str();
}

spk_status spk_server_destroy(spk_server srv) {
    if (!srv) return SPK_OK;
    if (srv->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stopping = true;
        }
        srv->cv.notify_all();
        srv->worker.join();
    }
    (void)hipSetDevice(srv->device);
    if (srv->stream) (void)hipStreamSynchronize(srv->stream);
    if (srv->tick_graph) (void)hipGraphExecDestroy(srv->tick_graph);
    for (Slot &sl : srv->slots)
        if (sl.ws) srv->pool.put(sl.ws);
    srv->pool.trim();
    void *dev_ptrs[] = {srv->d_counts, srv->d_tiles, srv->d_slots, srv->d_desc, srv->d_state, srv->d_status, srv->d_flags};
    for (void *p : dev_ptrs)
        if (p) (void)hipFree(p);
    void *host_ptrs[] = {srv->h_counts, srv->h_tiles, srv->h_slots, srv->h_desc, srv->h_state, srv->h_status, srv->h_flags};
    for (void *p : host_ptrs)
        if (p) (void)hipHostFree(p);
    if (srv->stream) (void)hipStreamDestroy(srv->stream);
    delete srv;
    return SPK_OK;
}

}  // extern "C"
