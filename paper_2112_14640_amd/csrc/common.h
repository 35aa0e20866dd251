// Shared device/host helpers for libdirac: complex arithmetic, storage precisions,
// lattice geometry, launch geometry and error plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/dirac.h"

namespace dirac {

// ---------------------------------------------------------------------------
// Complex numbers in registers
// ---------------------------------------------------------------------------
template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cmk(R a, R b) {
    return cx<R>{a, b};
}
template <typename R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) {
    return {a.re - b.re, a.im - b.im};
}
template <typename R>
__device__ __forceinline__ cx<R> cscale(R s, cx<R> a) {
    return {s * a.re, s * a.im};
}
// i * a
template <typename R>
__device__ __forceinline__ cx<R> cmuli(cx<R> a) {
    return {-a.im, a.re};
}
// acc += a * b
template <typename R>
__device__ __forceinline__ void cfma(cx<R>& acc, cx<R> a, cx<R> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename R>
__device__ __forceinline__ void cfma_conj(cx<R>& acc, cx<R> a, cx<R> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
}
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> cconj(cx<R> a) {
    return {a.re, -a.im};
}

// ---------------------------------------------------------------------------
// Storage precisions
// ---------------------------------------------------------------------------
struct bf16x2 {
    uint16_t re, im;
};

__device__ __forceinline__ float bf16_to_float(uint16_t h) {
    return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// Round to nearest, ties to even; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t float_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu) != 0u) return static_cast<uint16_t>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

// Load/store of one complex element of storage type S into/out of compute type R.
template <typename R, typename S>
struct io;

template <>
struct io<double, double2> {
    __device__ static __forceinline__ cx<double> ld(const double2* p) {
        double2 v = *p;
        return {v.x, v.y};
    }
    __device__ static __forceinline__ void st(double2* p, cx<double> v) { *p = make_double2(v.re, v.im); }
};
template <>
struct io<float, float2> {
    __device__ static __forceinline__ cx<float> ld(const float2* p) {
        float2 v = *p;
        return {v.x, v.y};
    }
    __device__ static __forceinline__ void st(float2* p, cx<float> v) { *p = make_float2(v.re, v.im); }
};
template <>
struct io<float, bf16x2> {
    __device__ static __forceinline__ cx<float> ld(const bf16x2* p) {
        uint32_t w = *reinterpret_cast<const uint32_t*>(p);
        return {__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u)};
    }
    __device__ static __forceinline__ void st(bf16x2* p, cx<float> v) {
        uint32_t w = static_cast<uint32_t>(float_to_bf16(v.re)) | (static_cast<uint32_t>(float_to_bf16(v.im)) << 16);
        *reinterpret_cast<uint32_t*>(p) = w;
    }
};
// Conversions used by casts and mixed-precision BLAS (double accumulate).
template <>
struct io<double, float2> {
    __device__ static __forceinline__ cx<double> ld(const float2* p) {
        float2 v = *p;
        return {static_cast<double>(v.x), static_cast<double>(v.y)};
    }
    __device__ static __forceinline__ void st(float2* p, cx<double> v) {
        *p = make_float2(static_cast<float>(v.re), static_cast<float>(v.im));
    }
};
template <>
struct io<double, bf16x2> {
    __device__ static __forceinline__ cx<double> ld(const bf16x2* p) {
        cx<float> f = io<float, bf16x2>::ld(p);
        return {static_cast<double>(f.re), static_cast<double>(f.im)};
    }
    __device__ static __forceinline__ void st(bf16x2* p, cx<double> v) {
        // double -> float (round to nearest) -> bf16 (round to nearest even)
        io<float, bf16x2>::st(p, cx<float>{static_cast<float>(v.re), static_cast<float>(v.im)});
    }
};
template <>
struct io<float, double2> {
    __device__ static __forceinline__ cx<float> ld(const double2* p) {
        double2 v = *p;
        return {static_cast<float>(v.x), static_cast<float>(v.y)};
    }
    __device__ static __forceinline__ void st(double2* p, cx<float> v) {
        *p = make_double2(static_cast<double>(v.re), static_cast<double>(v.im));
    }
};

// Precision bundles: S = vector storage, G = gauge storage, R = arithmetic.
struct PrecF64 {
    using S = double2;
    using G = double2;
    using R = double;
};
struct PrecF32 {
    using S = float2;
    using G = float2;
    using R = float;
};
struct PrecBF16 {
    using S = bf16x2;
    using G = float2;
    using R = float;
};

// ---------------------------------------------------------------------------
// Lattice geometry
// ---------------------------------------------------------------------------
struct Geom {
    int nx, ny, nz, nt;
    int64_t vol;
    int apbc;
};

struct Coord {
    int x, y, z, t;
};

__device__ __forceinline__ Coord site_coord(int64_t s, const Geom& g) {
    Coord c;
    int64_t q = s / g.nx;
    c.x = static_cast<int>(s - q * g.nx);
    int64_t q2 = q / g.ny;
    c.y = static_cast<int>(q - q2 * g.ny);
    int64_t q3 = q2 / g.nz;
    c.z = static_cast<int>(q2 - q3 * g.nz);
    c.t = static_cast<int>(q3);
    return c;
}

__device__ __forceinline__ int64_t site_index(int x, int y, int z, int t, const Geom& g) {
    return ((static_cast<int64_t>(t) * g.nz + z) * g.ny + y) * g.nx + x;
}

__device__ __forceinline__ int wrap(int v, int n) {
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

// Site traversal order of the stencil kernels.  The lattice is cut into xyz bricks of
// bx*by*bz sites; each brick column (the brick at every t) is walked with t slowest and x
// fastest inside the brick.  Consecutive threads therefore read neighbouring sites, the +-t
// neighbours of a brick slice are one brick slice (bx*by*bz sites) away in traversal order
// (well inside one XCD's L2, unlike a whole t-slice of the lattice), and rows of bx sites
// stay contiguous in memory.  Memory layout is unchanged; only the site each thread owns.
struct SiteOrder {
    int bx, by, bz;    // brick extents (divide nx, ny, nz)
    int nbx, nby;      // bricks along x and y
    int bslice;        // bx*by*bz
    int64_t column;    // bslice * nt sites per brick column
};

__device__ __forceinline__ int64_t ordered_site(int64_t i, const SiteOrder& o, const Geom& g) {
    const int64_t col = i / o.column;
    const int64_t r = i - col * o.column;
    const int t = static_cast<int>(r / o.bslice);
    int q = static_cast<int>(r - static_cast<int64_t>(t) * o.bslice);
    const int bxy = o.bx * o.by;
    const int lz = q / bxy;
    q -= lz * bxy;
    const int ly = q / o.bx;
    const int lx = q - ly * o.bx;
    const int cbx = static_cast<int>(col % o.nbx);
    const int64_t c2 = col / o.nbx;
    const int cby = static_cast<int>(c2 % o.nby);
    const int cbz = static_cast<int>(c2 / o.nby);
    return site_index(cbx * o.bx + lx, cby * o.by + ly, cbz * o.bz + lz, t, g);
}

// Brick extent along one axis: the whole axis when short, else 8 (or a divisor near it).
inline int brick_extent(int n) {
    if (n <= 12) return n;
    for (int b : {8, 12, 10, 6, 16, 4, 2})
        if (n % b == 0) return b;
    return n;
}

inline SiteOrder make_site_order(const Geom& g) {
    SiteOrder o;
    o.bx = brick_extent(g.nx);
    o.by = brick_extent(g.ny);
    o.bz = brick_extent(g.nz);
    o.nbx = g.nx / o.bx;
    o.nby = g.ny / o.by;
    o.bslice = o.bx * o.by * o.bz;
    o.column = static_cast<int64_t>(o.bslice) * g.nt;
    return o;
}

// XCD-aware block order: the hardware hands consecutive workgroups to the eight
// XCDs round-robin; remapping gives each XCD a contiguous range of logical blocks,
// so neighbouring sites (shared stencil reads) land in the same L2.  The launch
// grid must be a multiple of 8 blocks.
__device__ __forceinline__ int64_t logical_block() {
    const int64_t nb = gridDim.x;
    const int64_t per = nb >> 3;
    const int64_t b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

inline int64_t grid_blocks_x8(int64_t threads, int block) {
    int64_t nb = (threads + block - 1) / block;
    return (nb + 7) / 8 * 8;
}

// ---------------------------------------------------------------------------
// Host-side error plumbing
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);
int check_hip(hipError_t e, const char* what);

#define DIRAC_HIP(call)                                          \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return ::dirac::check_hip(e_, #call); \
    } while (0)

inline hipStream_t as_stream(void* s) {
    return reinterpret_cast<hipStream_t>(s);
}

inline size_t complex_bytes(dirac_prec p) {
    return p == DIRAC_FP64 ? 16 : (p == DIRAC_FP32 ? 8 : 4);
}
inline size_t gauge_complex_bytes(dirac_prec p) {
    return p == DIRAC_FP64 ? 16 : 8;
}

}  // namespace dirac
