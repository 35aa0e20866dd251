// Measurement probes (libdirac_probe.so, declared in dirac_probe.h): sustained copy bandwidth, FMA
// rate, and the stencils' row-gather access pattern without their arithmetic.  Not part of the
// method; self-contained (no code shared with the operator library).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dirac_probe.h"

namespace {

using u32x4 = unsigned int __attribute__((ext_vector_type(4)));

constexpr int kBad = -1, kHip = -3;

#define PROBE_HIP(call)                          \
    do {                                         \
        if ((call) != hipSuccess) return kHip;   \
    } while (0)

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

struct Lat {
    int nx, ny, nz, nt;
    int units;  // 16-byte units per site
};

// Row of logical tile T: 4 x 4 (y, z) blocks over the whole t range, the rows of a block innermost.
__device__ __forceinline__ int64_t gather_row(uint32_t T, const Lat& g) {
    const uint32_t rin = T % 16u, q = T / 16u;
    const uint32_t t = q % static_cast<uint32_t>(g.nt), blk = q / static_cast<uint32_t>(g.nt);
    const uint32_t nby = static_cast<uint32_t>(g.ny) / 4u;
    const uint32_t y = (blk % nby) * 4u + rin % 4u, z = (blk / nby) * 4u + rin / 4u;
    return (static_cast<int64_t>(t) * g.nz + z) * g.ny + y;
}

__device__ __forceinline__ int64_t step_row(int64_t row, int d, const Lat& g) {
    int y = static_cast<int>(row % g.ny);
    int z = static_cast<int>((row / g.ny) % g.nz);
    int t = static_cast<int>(row / (static_cast<int64_t>(g.ny) * g.nz));
    switch (d) {
        case 1: y = y + 1 == g.ny ? 0 : y + 1; break;
        case 2: y = y == 0 ? g.ny - 1 : y - 1; break;
        case 3: z = z + 1 == g.nz ? 0 : z + 1; break;
        case 4: z = z == 0 ? g.nz - 1 : z - 1; break;
        case 5: t = t + 1 == g.nt ? 0 : t + 1; break;
        case 6: t = t == 0 ? g.nt - 1 : t - 1; break;
        default: break;
    }
    return (static_cast<int64_t>(t) * g.nz + z) * g.ny + y;
}

constexpr int kGatherPer = 6;  // 16-byte units per thread and row

// One work-group per row: the rows' loads (own row, then +-y, +-z, +-t while d < nrows) are all issued
// before any is used.
template <int NROWS>
__global__ __launch_bounds__(512) void k_row_gather(const u32x4* __restrict__ in, u32x4* __restrict__ out, Lat g) {
    const uint32_t nb = gridDim.x, per = nb >> 3, b = blockIdx.x;
    const int64_t row = gather_row((b & 7u) * per + (b >> 3), g);
    const uint32_t row_units = static_cast<uint32_t>(g.nx * g.units);
    const uint32_t tid = threadIdx.x, nth = blockDim.x;
    u32x4 v[7][kGatherPer];
#pragma unroll
    for (int d = 0; d < 7; ++d) {
        const u32x4* src = in + step_row(row, d, g) * row_units;
#pragma unroll
        for (int k = 0; k < kGatherPer; ++k) {
            const uint32_t u = k * nth + tid;
            v[d][k] = u < row_units && d < NROWS ? src[u] : u32x4{0u, 0u, 0u, 0u};
        }
    }
    u32x4* dst = out + row * row_units;
#pragma unroll
    for (int k = 0; k < kGatherPer; ++k) {
        const uint32_t u = k * nth + tid;
        u32x4 acc = v[0][k];
#pragma unroll
        for (int d = 1; d < 7; ++d) acc ^= v[d][k];
        if (u < row_units) __builtin_nontemporal_store(acc, dst + u);
    }
}

template <typename F>
int time_launches(hipStream_t st, int reps, F launch, double* seconds) {
    hipEvent_t e0, e1;
    PROBE_HIP(hipEventCreate(&e0));
    PROBE_HIP(hipEventCreate(&e1));
    launch();  // warm-up
    PROBE_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) launch();
    PROBE_HIP(hipEventRecord(e1, st));
    PROBE_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    PROBE_HIP(hipEventElapsedTime(&ms, e0, e1));
    PROBE_HIP(hipEventDestroy(e0));
    PROBE_HIP(hipEventDestroy(e1));
    PROBE_HIP(hipGetLastError());
    *seconds = ms * 1e-3;
    return 0;
}

bool aligned16(const void* p) {
    return reinterpret_cast<uintptr_t>(p) % 16 == 0;
}

}  // namespace

extern "C" int dirac_probe_copy(const void* src, void* dst, size_t nbytes, int reps, double* bytes_per_s,
                                void* stream) {
    if (!src || !dst || !bytes_per_s || nbytes == 0 || nbytes % 16 != 0 || reps < 1 || !aligned16(src) ||
        !aligned16(dst))
        return kBad;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = static_cast<int64_t>(nbytes / 16);
    const dim3 grid(static_cast<unsigned>((n + 255) / 256));
    double sec = 0.0;
    const int rc = time_launches(st, reps, [&] {
        hipLaunchKernelGGL(k_copy16, grid, dim3(256), 0, st, static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n);
    }, &sec);
    if (rc) return rc;
    *bytes_per_s = 2.0 * static_cast<double>(nbytes) * reps / sec;  // read + write
    return 0;
}

extern "C" int dirac_probe_fma(int fp64, void* sink, double* flops_per_s, void* stream) {
    if (!sink || !flops_per_s || (fp64 != 0 && fp64 != 1)) return kBad;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    PROBE_HIP(hipGetDevice(&dev));
    PROBE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const dim3 grid(static_cast<unsigned>(cus * 16));  // 16 work-groups of 4 waves per CU
    const int reps = 5;
    double sec = 0.0;
    int rc;
    if (fp64 == 0)
        rc = time_launches(st, reps, [&] {
            hipLaunchKernelGGL(k_fma<float>, grid, dim3(256), 0, st, 0.999999f, 1e-7f, static_cast<float*>(sink));
        }, &sec);
    else
        rc = time_launches(st, reps, [&] {
            hipLaunchKernelGGL(k_fma<double>, grid, dim3(256), 0, st, 0.999999, 1e-7, static_cast<double*>(sink));
        }, &sec);
    if (rc) return rc;
    *flops_per_s = 2.0 * kChains * kFmaIters * 256.0 * grid.x * reps / sec;
    return 0;
}

extern "C" int dirac_probe_row_gather(const void* in, void* out, int nx, int ny, int nz, int nt, int site_bytes,
                                      int nrows, int reps, double* bytes_per_s, void* stream) {
    if (!in || !out || !bytes_per_s || reps < 1 || (nrows != 1 && nrows != 7) || nx < 1 || ny < 4 || nz < 4 ||
        nt < 1 || ny % 4 || nz % 4 ||
        site_bytes < 16 || site_bytes % 16 || !aligned16(in) || !aligned16(out))
        return kBad;
    const int64_t rows = static_cast<int64_t>(ny) * nz * nt;
    const int64_t row_units = static_cast<int64_t>(nx) * (site_bytes / 16);
    if (rows % 8 || rows > (int64_t{1} << 31) - 1 || row_units > 512 * kGatherPer) return kBad;
    int threads = static_cast<int>((row_units + kGatherPer - 1) / kGatherPer);
    threads = (threads + 63) / 64 * 64;
    const Lat g{nx, ny, nz, nt, site_bytes / 16};
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double sec = 0.0;
    const auto kern = nrows == 7 ? k_row_gather<7> : k_row_gather<1>;
    const int rc = time_launches(st, reps, [&] {
        hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(rows)), dim3(threads), 0, st,
                           static_cast<const u32x4*>(in), static_cast<u32x4*>(out), g);
    }, &sec);
    if (rc) return rc;
    *bytes_per_s = 2.0 * static_cast<double>(rows * row_units * 16) * reps / sec;
    return 0;
}
