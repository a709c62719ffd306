// Internal types and constants shared by the host runtime (spk_api.cpp,
// spk_server.cpp) and the gfx950 kernels.  The launchers that start the
// kernels are declared in spk_launch.h.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

struct spk_ctx_s;

namespace spk {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64s)
constexpr int kTileRows = 256;     // rows per SpMV tile
constexpr int kMaxGrid = 8192;     // cap on workgroups of any grid-stride launch
constexpr int kNumXcd = 8;         // MI355X: 8 XCDs, workgroups dispatched round-robin
// Device scratch of the allocation-free solve (one array per GPU, held until
// the process ends): solve state, reduction partials and three FP64 vectors.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;

enum Stop : int32_t {
    STOP_RUNNING = 0,
    STOP_CONVERGED = 1,
    STOP_MAX_ITERS = 2,
    STOP_BREAKDOWN = 3,
    STOP_NON_FINITE = 4
};

// Reduction sites: each owns an arrival counter and a partials slab.
// SITE_FCG: the fused CG step's two partial sets (p.q, r.q, q.q, r.r; one set
// per iteration parity), slabs 4 * parity + j from the site's start.
enum Site : int { SITE_INIT = 0, SITE_PQ = 1, SITE_RR = 2, SITE_TRUE = 3, SITE_FCG = 4, SITE_COUNT = 7 };
constexpr int kSiteWidth = 3;      // values reduced at once per site (max)

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
    void *x;              // solution vector of this solve (FP64 x, or FP32 d of an inner solve)
    double *hist;         // optional ||r_k|| history
    int64_t hist_cap;
};

// Vector pairs of the fused CG loop: step k reads buffer (k + 1) & 1 of each
// pair and writes buffer k & 1; the initial residual goes to buffer 1.
template <typename T>
struct FcgBufs {
    T *r[2], *p[2], *q[2];
};

// Result of a persistent mixed-precision solve (written by workgroup 0).
struct PersistResult {
    int64_t inner, outer;   // inner iterations in all, refinement steps
    double rnorm, bnorm;    // last ||b - A x|| (FP64) and ||b||
    int32_t stop;
};

// Arguments of a persistent solve (matrix fields filled by the launcher).
struct PersistSolve {
    int64_t n, nnz;
    const void *rp, *ci, *va, *va64;
    const double *b;
    double *x;
    FcgBufs<double> f64;   // FP64 solve
    FcgBufs<float> f32;    // mixed: inner vectors
    float *d32;            // mixed: inner correction
    SolveState *st;        // FP64 solve: the state the host reads
    PersistResult *res;    // mixed: the result
    double *partials;
    unsigned *bar;
    uint64_t spin_ticks;
    double tau, tau_in;
    int64_t max_iters, max_outer;
    double *hist;
    int64_t hist_cap;
    int remap, nt, true_residual;
};

// Restarted GMRES: the small per-solve arrays (device memory, one per plan).
constexpr int kMaxKrylov = 32;   // largest restart length m
struct GmresState {
    double H[(kMaxKrylov + 1) * kMaxKrylov];   // rotated Hessenberg, H[i * kMaxKrylov + j]
    double Hu[(kMaxKrylov + 1) * kMaxKrylov];  // the same columns unrotated (A Q = Q Hu)
    double cs[kMaxKrylov], sn[kMaxKrylov];     // Givens rotations
    double g[kMaxKrylov + 1];                  // rotated right-hand side beta e_0
    double y[kMaxKrylov];                      // solution of R y = g
    double b[kMaxKrylov + 1];                  // first pass: q_t . w (t < j), u_j . w
    double a[kMaxKrylov + 1];                  // candidate u_j = Q_j a + nu q_j: its components along Q_j
    double h[kMaxKrylov + 1];                  // column j before the delayed correction
    double d[kMaxKrylov + 1];                  // u_{j+1} = w / nu - sum d_t q_t
    double nu;                                 // norm of the candidate's part orthogonal to Q_j
    int32_t used;                              // columns built in this cycle
    int32_t cycle_done;                        // nonzero: later kernels of the cycle return at once
};

// Launch shape of the SpMV family (shared by every SpMV-based kernel).
struct SpmvTune {
    int kind;        // 0 = LDS-staged row tiles, 1 = lanes-per-row vector kernel
    int lanes_log2;  // vector kernel: log2(lanes per row)
    int grid;        // workgroups
    int xcd_remap;   // 1 = contiguous tile ranges per XCD
    int nt;          // 1 = non-temporal loads for the matrix value stream
    int pf;          // LDS tiles: 1 = the next tile's row pointers load while this tile's entries stream in
    int bpc;         // workgroups per CU the grid was sized for
    int codes = 0;   // LDS tiles: 1 = read the matrix's one-byte column codes (CsrDev::codes)
    int pack = 0;    // with codes: 1 = read the packed row pointers (CsrDev::rowpack)
    int cus = 0;     // compute units of the device (0 = unknown: every workgroup walks tiles)
};

// Device CSR view with runtime-typed arrays.
struct CsrDev {
    int64_t n_rows, n_cols, nnz;
    int ptr_t, idx_t, val_t;   // spk_itype / spk_dtype codes
    const void *rp, *ci, *va;
    // Optional one-byte column codes (null when absent): byte k names entry k's
    // column offset from its row, c - i, in a table of kCodeDict int64 offsets
    // stored in the kCodeDict * 8 bytes just before the codes.
    const void *codes = nullptr;
    // Optional packed row pointers (null when absent; only with codes): the
    // int64 first entry of every 256-row tile (tiles + 1 values), followed
    // directly by one uint16 per row, its first entry less its tile's.
    const void *rowpack = nullptr;
    // The longest row's entry count (measured when the plan validates A; 0 =
    // unknown).  Above kLongRow the row tiles sum such rows with the whole
    // workgroup (host side only: it sets the kernels' long-row argument).
    int64_t max_row = 0;
};

constexpr int kLongRow = 256;   // rows longer than this are summed by a whole workgroup

constexpr int kCodeDict = 256;    // distinct column offsets a code table holds
constexpr int kCodeSlots = 1024;  // plan-time hash table of distinct offsets (power of two)

// Byte sizes of the plan's code buffer: the offset table, the codes (rounded
// to 16 bytes), then the packed row pointers (tiles + 1 int64, n uint16).
inline size_t code_bytes(int64_t nnz) { return (static_cast<size_t>(nnz) + 15) & ~size_t(15); }
inline size_t code_buffer_bytes(int64_t n_rows, int64_t nnz) {
    const size_t tiles = static_cast<size_t>((n_rows + kTileRows - 1) / kTileRows);
    return sizeof(int64_t) * kCodeDict + code_bytes(nnz) + sizeof(int64_t) * (tiles + 1) +
           ((sizeof(uint16_t) * static_cast<size_t>(n_rows) + 15) & ~size_t(15));
}

// Validation flag bits (set by the GPU check, order resolved on the host).
enum : unsigned { VFLAG_BAD_FIRST = 1u, VFLAG_DECREASING = 2u, VFLAG_BAD_LAST = 4u, VFLAG_BAD_COLUMN = 8u,
                  VFLAG_UNSORTED = 16u };

}  // namespace spk

// ==== batched serving ==========================================================
namespace spk {

// Per-slot life cycle, advanced on the device once per tick.
enum Phase : int32_t {
    PH_FREE = 0,     // slot unused
    PH_OUTER = 1,    // refinement residual r = b - A x (FP64) this tick
    PH_INNER = 2,    // CG iterations on A d = r (FP32 with FP64 dots, or FP64)
    PH_CORRECT = 3,  // x += d this tick
    PH_ZEROX = 4,    // b == 0: x = 0 this tick
    PH_DONE = 5      // finished; waiting for the host to retire it
};

// Per-slot partial-sum sites (kPartSites doubles per tile).
enum : int { PART_PQ = 0, PART_RR = 1, PART_OUT = 2 /* 3 sites: r.r, r32.r32, b.b */, kPartSites = 5 };

// Written by the host at admission; read-only on the device.
struct SlotDesc {
    int64_t n, nnz, tiles;
    const int32_t *rp, *ci;
    const double *va64;     // the request's FP64 values
    const float *va32;      // rounded copy (slot workspace)
    const double *b;
    double *x;
    float *r, *p, *q, *d;          // slot workspace of an FP32-inner request
    double *r64, *p64, *q64, *d64; // slot workspace of an FP64 request
    double *part;                  // slot workspace: kPartSites * tiles
    double tau, tau_in;
    int64_t max_iters, max_outer;
    int32_t stage;          // 1: values and columns 16-byte aligned, tiles staged in LDS by DMA
    int32_t fp64;           // 1: the inner CG runs in FP64 on the caller's values (no FP32 copy)
};

// Device-resident per-slot scalars.
struct SlotState {
    double rho[4];
    double thresh_in, bnorm, rnorm, alpha, beta;
    int64_t iter_in, iters, outer;
    int32_t phase, next_phase, stop_in, stop;
};

// Compact per-slot record the host polls after each batch of ticks.
struct SlotStatus {
    int32_t phase, stop;
    int64_t iters, outer;
    double rnorm, bnorm;
};

// Device tables of one server: counts plus tile and slot lists.
struct BatchDev {
    const int32_t *counts;   // [0] live tiles, [1] live slots
    const int2 *tiles;       // (slot, local tile)
    const int32_t *slots;    // live slot ids
    const SlotDesc *desc;
    SlotState *state;
    SlotStatus *status;
    int tile_grid, slot_grid;
    int remap;   // tile order of the tile launches (TileIter: 0 round-robin, 1 contiguous eighths per XCD)
    int nt;      // 1: non-temporal loads of the matrix stream
};

}  // namespace spk
