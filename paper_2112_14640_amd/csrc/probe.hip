// Measurement probes: the sustained copy bandwidth and FMA rate of the device, the measured
// denominators next to the published peaks in the roofline figures.  Not part of the method.
#include <cmath>

#include "common.h"

namespace dirac {

namespace {

using u32x4 = unsigned int __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// CHAINS independent FMA chains per thread, ITERS steps each: 2 * CHAINS * ITERS flops per thread.
constexpr int kChains = 16;
constexpr int kFmaIters = 2048;

template <typename T>
__global__ __launch_bounds__(256) void k_fma(T x, T y, T* __restrict__ sink) {
    T a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = static_cast<T>(threadIdx.x + c);
    for (int it = 0; it < kFmaIters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) a[c] = fma(a[c], x, y);
    }
    T s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += a[c];
    if (s == static_cast<T>(-1.25)) sink[0] = s;  // keeps the chains alive; never true for the inputs used
}

template <typename F>
int time_launches(hipStream_t st, int reps, F launch, double* seconds) {
    hipEvent_t e0, e1;
    DIRAC_HIP(hipEventCreate(&e0));
    DIRAC_HIP(hipEventCreate(&e1));
    launch();  // warm-up
    DIRAC_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) launch();
    DIRAC_HIP(hipEventRecord(e1, st));
    DIRAC_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    DIRAC_HIP(hipEventElapsedTime(&ms, e0, e1));
    DIRAC_HIP(hipEventDestroy(e0));
    DIRAC_HIP(hipEventDestroy(e1));
    *seconds = ms * 1e-3;
    return DIRAC_OK;
}

}  // namespace

}  // namespace dirac

using namespace dirac;

extern "C" int dirac_probe_copy(const void* src, void* dst, size_t nbytes, int reps, double* bytes_per_s,
                                void* stream) {
    if (!src || !dst || !bytes_per_s || nbytes == 0 || nbytes % 16 != 0 || reps < 1)
        return fail(DIRAC_EINVAL, "dirac_probe_copy: need buffers, a byte count that is a positive multiple of 16 "
                                  "and reps >= 1");
    if (reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return fail(DIRAC_EINVAL, "dirac_probe_copy: buffers must be 16-byte aligned");
    hipStream_t st = as_stream(stream);
    const int64_t n = static_cast<int64_t>(nbytes / 16);
    const dim3 grid(static_cast<unsigned>((n + 255) / 256));
    double sec = 0.0;
    int rc = time_launches(st, reps, [&] {
        hipLaunchKernelGGL(k_copy16, grid, dim3(256), 0, st, static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n);
    }, &sec);
    if (rc) return rc;
    DIRAC_HIP(hipGetLastError());
    *bytes_per_s = 2.0 * static_cast<double>(nbytes) * reps / sec;  // read + write
    return DIRAC_OK;
}

extern "C" int dirac_probe_fma(dirac_prec prec, void* sink, double* flops_per_s, void* stream) {
    if (!sink || !flops_per_s) return fail(DIRAC_EINVAL, "dirac_probe_fma: need a sink buffer and an output");
    if (prec != DIRAC_FP32 && prec != DIRAC_FP64) return fail(DIRAC_EINVAL, "dirac_probe_fma: FP32 or FP64");
    hipStream_t st = as_stream(stream);
    int dev = 0, cus = 0;
    DIRAC_HIP(hipGetDevice(&dev));
    DIRAC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const dim3 grid(static_cast<unsigned>(cus * 16));  // 16 work-groups of 4 waves per CU
    const int reps = 5;
    double sec = 0.0;
    int rc;
    if (prec == DIRAC_FP32)
        rc = time_launches(st, reps, [&] {
            hipLaunchKernelGGL(k_fma<float>, grid, dim3(256), 0, st, 0.999999f, 1e-7f, static_cast<float*>(sink));
        }, &sec);
    else
        rc = time_launches(st, reps, [&] {
            hipLaunchKernelGGL(k_fma<double>, grid, dim3(256), 0, st, 0.999999, 1e-7, static_cast<double*>(sink));
        }, &sec);
    if (rc) return rc;
    DIRAC_HIP(hipGetLastError());
    *flops_per_s = 2.0 * kChains * kFmaIters * 256.0 * grid.x * reps / sec;
    return DIRAC_OK;
}
