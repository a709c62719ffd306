// Library-owned scratch memory for the allocation-free solve entry point
// (spk_solve_noalloc).  The workspace of one FP64 CG solve (state, reduction
// partials, r, p, q) lives in a file-scope device array of fixed size, so a
// caller that must not allocate device memory (graph capture, tight serving
// loops, harnesses that forbid hipMalloc) can still run a solve.
//
// Host code never passes the array's name to a kernel: in host code that
// name is only a stand-in.  The device address of each GPU's copy is looked
// up once per device with hipGetSymbolAddress (at context creation, with the
// device current) and kept; every kernel argument, fill and copy uses that
// address.
#include "spk_internal.h"
#include "spk_launch.h"

#include <mutex>

static __device__ __align__(256) unsigned char scratch[spk::kNoallocScratchBytes];

namespace spk {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

__global__ __launch_bounds__(kBlock) void k_fill_zero(uint4 *__restrict__ p, int64_t n16) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

hipError_t noalloc_scratch_setup(int device, void **addr) {
    *addr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_done[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_err[device] = e;
        g_addr[device] = e == hipSuccess ? p : nullptr;
        g_done[device] = true;
    }
    *addr = g_addr[device];
    return g_err[device];
}

hipError_t launch_fill_zero(void *p, size_t bytes, int grid, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if ((reinterpret_cast<uintptr_t>(p) & 15) || (bytes & 15)) return hipErrorInvalidValue;
    const int64_t n16 = static_cast<int64_t>(bytes / 16);
    const int64_t want = (n16 + kBlock - 1) / kBlock;
    const int g = static_cast<int>(want < grid ? (want < 1 ? 1 : want) : grid);
    hipLaunchKernelGGL(k_fill_zero, dim3(g), dim3(kBlock), 0, s, static_cast<uint4 *>(p), n16);
    return hipGetLastError();
}

}  // namespace spk
