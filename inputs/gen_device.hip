// Seeded synthetic inputs generated on the GPU (for instances too large to
// build on the host and copy, e.g. stencil7 N = 1048: 8e9 stored entries).
// Same definitions as gen.c (counter-based SplitMix64 draws, stencil7
// pattern, diagonal = sum of |off-diagonals| in ascending column order +
// delta), so the device and host generators produce bit-identical arrays.
// Holds no solver arithmetic.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ULL;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t hash3(uint64_t seed, uint64_t stream, uint64_t ctr) {
    const uint64_t k = mix64(seed * kGolden + stream);
    return mix64(k + (ctr + 1) * kGolden);
}

__device__ __forceinline__ double unif_f64(uint64_t seed, uint64_t stream, uint64_t ctr) {
    const uint64_t h = hash3(seed, stream, ctr);
    const double u = static_cast<double>(h >> 11) * 0x1.0p-53;
    return 2.0 * u - 1.0;
}

__device__ __forceinline__ double unif_f32x(uint64_t seed, uint64_t stream, uint64_t ctr) {
    const uint64_t h = hash3(seed, stream, ctr);
    return static_cast<double>(static_cast<int64_t>(h >> 40)) * 0x1.0p-23 - 1.0;
}

__device__ __forceinline__ double offdiag(uint64_t seed, uint64_t edge, int f32x) {
    return f32x ? unif_f32x(seed, 0, edge) : unif_f64(seed, 0, edge);
}

__device__ __forceinline__ double round_up_f32(double d) {
    float f = static_cast<float>(d);
    if (static_cast<double>(f) < d) f = nextafterf(f, __builtin_inff());
    return static_cast<double>(f);
}

// Entries stored before row i: 7 i minus the missing neighbours of rows j < i.
__device__ __forceinline__ int64_t stencil7_row_start(int64_t i, int64_t N) {
    const int64_t N2 = N * N;
    const int64_t x = i % N, y = (i / N) % N, z = i / N2;
    const int64_t xlo = (i + N - 1) / N;                 // rows j < i with x_j = 0
    const int64_t xhi = i / N;                           // x_j = N-1
    const int64_t inplane = x + N * y;
    const int64_t ylo = N * z + (inplane < N ? inplane : N);
    int64_t t = x + N * (y - (N - 1));
    t = t < 0 ? 0 : (t > N ? N : t);
    const int64_t yhi = N * z + t;                       // y_j = N-1
    const int64_t zlo = i < N2 ? i : N2;                 // z_j = 0
    const int64_t zhi = i > N2 * (N - 1) ? i - N2 * (N - 1) : 0;   // z_j = N-1
    return 7 * i - xlo - xhi - ylo - yhi - zlo - zhi;
}

template <typename V>
__global__ __launch_bounds__(256) void k_stencil7(int64_t N, uint64_t seed, double delta, int f32x, int64_t *rp,
                                                  int32_t *col, V *val) {
    const int64_t n = N * N * N, s1 = N, s2 = N * N;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) {
        const int64_t x = i % N, y = (i / N) % N, z = i / s2;
        int64_t cj[7];
        double cv[7];
        int m = 0, dpos = 0;
        if (z > 0) { cj[m] = i - s2; cv[m] = offdiag(seed, 3 * static_cast<uint64_t>(i - s2) + 2, f32x); ++m; }
        if (y > 0) { cj[m] = i - s1; cv[m] = offdiag(seed, 3 * static_cast<uint64_t>(i - s1) + 1, f32x); ++m; }
        if (x > 0) { cj[m] = i - 1; cv[m] = offdiag(seed, 3 * static_cast<uint64_t>(i - 1) + 0, f32x); ++m; }
        dpos = m;
        cj[m] = i;
        cv[m] = 0.0;
        ++m;
        if (x < N - 1) { cj[m] = i + 1; cv[m] = offdiag(seed, 3 * static_cast<uint64_t>(i) + 0, f32x); ++m; }
        if (y < N - 1) { cj[m] = i + s1; cv[m] = offdiag(seed, 3 * static_cast<uint64_t>(i) + 1, f32x); ++m; }
        if (z < N - 1) { cj[m] = i + s2; cv[m] = offdiag(seed, 3 * static_cast<uint64_t>(i) + 2, f32x); ++m; }
        double d = 0.0;
        for (int t = 0; t < m; ++t)
            if (t != dpos) d = d + fabs(cv[t]);
        d = d + delta;
        cv[dpos] = f32x ? round_up_f32(d) : d;
        const int64_t k0 = stencil7_row_start(i, N);
        for (int t = 0; t < m; ++t) {
            col[k0 + t] = static_cast<int32_t>(cj[t]);
            val[k0 + t] = static_cast<V>(cv[t]);
        }
        rp[i] = k0;
        if (i == n - 1) rp[n] = k0 + m;
    }
}

__global__ __launch_bounds__(256) void k_rhs(int64_t n, uint64_t seed, uint64_t stream, double *b) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride)
        b[i] = unif_f64(seed, stream, static_cast<uint64_t>(i));
}

}  // namespace

extern "C" {

// stencil7(N) into device arrays: rp int64[N^3 + 1], col int32[7N^3 - 6N^2],
// val FP64 (val_f32 = 0) or FP32 (val_f32 = 1, only meaningful with f32x = 1).
// N^3 must be below 2^31 (int32 columns).  Returns a hipError_t code.
int gen_dev_stencil7(int64_t N, uint64_t seed, double delta, int f32x, void *rp, void *col, void *val, int val_f32,
                     void *stream) {
    if (N < 1 || N * N * N >= (int64_t(1) << 31)) return static_cast<int>(hipErrorInvalidValue);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int grid = 4096;
    if (val_f32)
        hipLaunchKernelGGL(k_stencil7<float>, dim3(grid), dim3(256), 0, s, N, seed, delta, f32x,
                           static_cast<int64_t *>(rp), static_cast<int32_t *>(col), static_cast<float *>(val));
    else
        hipLaunchKernelGGL(k_stencil7<double>, dim3(grid), dim3(256), 0, s, N, seed, delta, f32x,
                           static_cast<int64_t *>(rp), static_cast<int32_t *>(col), static_cast<double *>(val));
    return static_cast<int>(hipGetLastError());
}

// b_i = uniform[-1,1) draw (seed, stream, i), FP64.
int gen_dev_vec(int64_t n, uint64_t seed, uint64_t stream, void *b, void *s) {
    hipLaunchKernelGGL(k_rhs, dim3(4096), dim3(256), 0, static_cast<hipStream_t>(s), n, seed, stream,
                       static_cast<double *>(b));
    return static_cast<int>(hipGetLastError());
}

}  // extern "C"
