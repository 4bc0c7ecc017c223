// Roofline probes: the HBM bandwidth and matrix-core rates this GPU achieves, measured with the
// simplest kernels that can reach them, so that the solver's kernels can be read against measured
// ceilings as well as the datasheet's (HBM 8 TB/s; FP64 matrix 78.6 TFLOP/s, FP32 matrix 157.3).
//
//   copy   b = a                    2 x bytes moved per pass
//   triad  a = b + s c (FP64)       3 x bytes
//   read   sum of a (one partial per workgroup)
//   mfma   register-resident chains of v_mfma_f64_16x16x4 / v_mfma_f32_16x16x4 on every SIMD
//
// The bandwidth kernels stride over the buffers with 16-byte loads, four independent ones per
// thread and pass, consecutive lanes on consecutive addresses.
#include <algorithm>
#include <new>
#include <stdexcept>
#include <string>

#include "kernels.h"

namespace scg {

constexpr int PB_U = 4;   // 16-byte elements per thread and pass

__global__ __launch_bounds__(256) void probe_copy_kernel(const double2* __restrict__ a, double2* __restrict__ b, int64_t n) {
    const int64_t step = (int64_t)gridDim.x * 256 * PB_U;
    for (int64_t base = (int64_t)blockIdx.x * 256 * PB_U + threadIdx.x; base < n; base += step) {
        double2 v[PB_U];
#pragma unroll
        for (int u = 0; u < PB_U; u++) {
            const int64_t i = base + u * 256;
            if (i < n) v[u] = a[i];
        }
#pragma unroll
        for (int u = 0; u < PB_U; u++) {
            const int64_t i = base + u * 256;
            if (i < n) b[i] = v[u];
        }
    }
}

__global__ __launch_bounds__(256) void probe_triad_kernel(double2* __restrict__ a, const double2* __restrict__ b,
                                                          const double2* __restrict__ c, double s, int64_t n) {
    const int64_t step = (int64_t)gridDim.x * 256 * PB_U;
    for (int64_t base = (int64_t)blockIdx.x * 256 * PB_U + threadIdx.x; base < n; base += step) {
        double2 x[PB_U], y[PB_U];
#pragma unroll
        for (int u = 0; u < PB_U; u++) {
            const int64_t i = base + u * 256;
            if (i < n) {
                x[u] = b[i];
                y[u] = c[i];
            }
        }
#pragma unroll
        for (int u = 0; u < PB_U; u++) {
            const int64_t i = base + u * 256;
            if (i < n) a[i] = make_double2(x[u].x + s * y[u].x, x[u].y + s * y[u].y);
        }
    }
}

__global__ __launch_bounds__(256) void probe_read_kernel(const double2* __restrict__ a, int64_t n, double* part) {
    __shared__ double lds[256 / SCG_WAVE];
    const int64_t step = (int64_t)gridDim.x * 256 * PB_U;
    double s = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * 256 * PB_U + threadIdx.x; base < n; base += step) {
        double2 v[PB_U];
#pragma unroll
        for (int u = 0; u < PB_U; u++) {
            const int64_t i = base + u * 256;
            v[u] = i < n ? a[i] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < PB_U; u++) s += v[u].x + v[u].y;
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T>
struct ProbeMfma;
template <>
struct ProbeMfma<double> {
    using V4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    __device__ static inline V4 step(double a, double b, V4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
template <>
struct ProbeMfma<float> {
    using V4 = __attribute__((__vector_size__(4 * sizeof(float)))) float;
    __device__ static inline V4 step(float a, float b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

// PB_CHAINS independent accumulator chains per wavefront, so that the matrix core never waits on the
// previous product of a chain; one value per workgroup is written so the work cannot be dropped
constexpr int PB_CHAINS = 8;
template <typename T>
__global__ __launch_bounds__(256) void probe_mfma_kernel(int iters, T a0, double* out) {
    using M = ProbeMfma<T>;
    typename M::V4 acc[PB_CHAINS];
#pragma unroll
    for (int c = 0; c < PB_CHAINS; c++)
#pragma unroll
        for (int q = 0; q < 4; q++) acc[c][q] = 0;
    const T a = a0 + (T)(threadIdx.x % 64) * (T)1e-3, b = a0 - (T)(threadIdx.x % 64) * (T)1e-3;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int c = 0; c < PB_CHAINS; c++) acc[c] = M::step(a, b, acc[c]);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < PB_CHAINS; c++)
#pragma unroll
        for (int q = 0; q < 4; q++) s += (double)acc[c][q];
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

namespace {
// hipEvent pair around `reps` launches after one untimed launch; milliseconds per launch
template <typename F>
double time_launches(hipStream_t s, int reps, F launch) {
    launch();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; r++) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) throw std::runtime_error(std::string("probe: ") + hipGetErrorString(e));
    return (double)ms / reps;
}
struct ProbeBuf {
    void* p = nullptr;
    explicit ProbeBuf(size_t n) {
        if (hipMalloc(&p, n) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            throw std::bad_alloc();
        }
    }
    ~ProbeBuf() {
        if (p) (void)hipFree(p);
    }
};
}  // namespace

double probe_bandwidth(int kind, int64_t bytes, int reps, hipStream_t s) {
    if (kind < 0 || kind > 2) throw std::invalid_argument("probe_bandwidth: kind 0 (copy), 1 (triad) or 2 (read)");
    if (bytes < (1 << 20) || reps < 1) throw std::invalid_argument("probe_bandwidth: bytes >= 1 MiB and reps >= 1");
    const int64_t n = bytes / 16;   // 16-byte elements per buffer
    const size_t nb = (size_t)n * 16;
    const unsigned grid = 8192;
    double ms = 0.0, moved = 0.0;
    if (kind == 0) {
        ProbeBuf a(nb), b(nb);
        (void)hipMemsetAsync(a.p, 0, nb, s);
        ms = time_launches(s, reps, [&]() {
            hipLaunchKernelGGL(probe_copy_kernel, dim3(grid), dim3(256), 0, s, (const double2*)a.p, (double2*)b.p, n);
        });
        moved = 2.0 * nb;
    } else if (kind == 1) {
        ProbeBuf a(nb), b(nb), c(nb);
        (void)hipMemsetAsync(b.p, 0, nb, s);
        (void)hipMemsetAsync(c.p, 0, nb, s);
        ms = time_launches(s, reps, [&]() {
            hipLaunchKernelGGL(probe_triad_kernel, dim3(grid), dim3(256), 0, s, (double2*)a.p, (const double2*)b.p, (const double2*)c.p,
                               0.5, n);
        });
        moved = 3.0 * nb;
    } else {
        ProbeBuf a(nb), part(grid * sizeof(double));
        (void)hipMemsetAsync(a.p, 0, nb, s);
        ms = time_launches(s, reps, [&]() {
            hipLaunchKernelGGL(probe_read_kernel, dim3(grid), dim3(256), 0, s, (const double2*)a.p, n, (double*)part.p);
        });
        moved = (double)nb;
    }
    return moved / (ms * 1e-3) / 1e9;
}

double probe_mfma(int dtype, int iters, hipStream_t s) {
    if (dtype < 0 || dtype > 1) throw std::invalid_argument("probe_mfma: dtype 0 (FP64) or 1 (FP32)");
    if (iters < 1) throw std::invalid_argument("probe_mfma: iters >= 1");
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) throw std::runtime_error(std::string("probe_mfma: ") + hipGetErrorString(e));
    // four workgroups of four wavefronts per compute unit: four wavefronts per SIMD
    const unsigned grid = (unsigned)std::max(1, ncu) * 4;
    ProbeBuf out(grid * sizeof(double));
    double ms = 0.0;
    if (dtype == 0)
        ms = time_launches(s, 3, [&]() {
            hipLaunchKernelGGL(probe_mfma_kernel<double>, dim3(grid), dim3(256), 0, s, iters, 0.5, (double*)out.p);
        });
    else
        ms = time_launches(s, 3, [&]() {
            hipLaunchKernelGGL(probe_mfma_kernel<float>, dim3(grid), dim3(256), 0, s, iters, 0.5f, (double*)out.p);
        });
    // 2 * 16 * 16 * 4 flops per instruction and wavefront
    const double flops = (double)grid * 4.0 * PB_CHAINS * (double)iters * 2048.0;
    return flops / (ms * 1e-3) / 1e12;
}

}  // namespace scg
