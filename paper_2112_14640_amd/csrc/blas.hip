// Multi-RHS BLAS-1 and the fused Krylov update kernels (Sec. 3: norms, dot products,
// "incr"/"anti" multiply-adds, casts, gamma_5 / epsilon).
//
// A vector is `nrows` rows of `nv` complex numbers (the right-hand-side index is fastest).
// Arithmetic is FP64 whatever the storage precision, and so is every accumulation.
// Reductions are two-pass and deterministic: a fixed grid of kReduceBlocks blocks, each
// block handles rows blockIdx + k * gridDim in a fixed order and reduces per RHS through
// LDS in a fixed order, then one block per output value adds the block partials with a
// fixed tree.  Repeated runs give bitwise identical results.
#include <algorithm>
#include <initializer_list>
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace dirac {

namespace {

template <typename T>
struct Tag {
    using type = T;
};

template <typename F>
int with_prec(dirac_prec p, F&& f) {
    switch (p) {
        case DIRAC_FP64: return f(Tag<double2>{});
        case DIRAC_FP32: return f(Tag<float2>{});
        case DIRAC_BF16: return f(Tag<bf16x2>{});
    }
    return DIRAC_EINVAL;
}

template <typename S>
__device__ __forceinline__ cx<double> ldd(const S* p) {
    return io<double, S>::ld(p);
}
template <typename S>
__device__ __forceinline__ void std_(S* p, cx<double> v) {
    io<double, S>::st(p, v);
}

// The value a store of v into storage S leaves behind, without touching memory.
template <typename S>
__device__ __forceinline__ cx<double> stored_value(cx<double> v) {
    S tmp;
    io<double, S>::st(&tmp, v);
    return io<double, S>::ld(&tmp);
}

// Packs: VW consecutive complex elements of one row (consecutive right-hand sides) moved with a single
// 4-, 8- or 16-byte access, so that FP32 and BF16 vectors stream with the same 16-byte lane accesses
// as FP64 ones.  VW = 16 bytes / the widest element of a kernel's vectors (1 when that does not divide
// nv or a pointer is not aligned to the pack).
using pk_u32x2 = unsigned int __attribute__((ext_vector_type(2)));
using pk_u32x4 = unsigned int __attribute__((ext_vector_type(4)));
template <int BYTES>
struct RawT;
template <>
struct RawT<4> {
    using T = unsigned int;
};
template <>
struct RawT<8> {
    using T = pk_u32x2;
};
template <>
struct RawT<16> {
    using T = pk_u32x4;
};
template <typename S, int VW>
struct Pack {
    S e[VW];
};

template <int VW, typename S>
__device__ __forceinline__ void ldp(const S* p, cx<double> (&v)[VW]) {
    using T = typename RawT<sizeof(S) * VW>::T;
    const Pack<S, VW> pk = __builtin_bit_cast(Pack<S, VW>, *reinterpret_cast<const T*>(p));
#pragma unroll
    for (int i = 0; i < VW; ++i) v[i] = ldd(&pk.e[i]);
}

template <int VW, typename S>
__device__ __forceinline__ void stp(S* p, const cx<double> (&v)[VW]) {
    using T = typename RawT<sizeof(S) * VW>::T;
    Pack<S, VW> pk;
#pragma unroll
    for (int i = 0; i < VW; ++i) std_(&pk.e[i], v[i]);
    *reinterpret_cast<T*>(p) = __builtin_bit_cast(T, pk);
}

template <typename... S>
constexpr int pack_width() {
    constexpr size_t m = std::max({sizeof(S)...});
    return static_cast<int>(16 / m);
}

inline bool pack_ok(int vw, int nv, std::initializer_list<const void*> ptrs) {
    if (vw <= 1) return true;
    if (nv % vw != 0) return false;
    for (const void* p : ptrs)
        if (reinterpret_cast<uintptr_t>(p) % 16 != 0) return false;
    return true;
}

// Packed row lanes: rows of nvp = nv / VW packs; thread (roff, pk) handles pack pk of row
// blockIdx * rpb + roff + k * gridDim * rpb.
struct PackLane {
    int nvp, rpb, roff, pk;
};
__device__ __forceinline__ PackLane pack_lane(int nvp) {
    PackLane r;
    r.nvp = nvp;
    r.rpb = kReduceThreads / nvp;
    r.roff = threadIdx.x / nvp;
    r.pk = threadIdx.x - r.roff * nvp;
    return r;
}

// Per-block per-RHS partial sums of W values for each of the VW elements of a thread's pack, written as
// partial[(block * W + w) * nv + rhs] (the layout finalize() reads); fixed summation order.
template <int W, int VW>
__device__ __forceinline__ void block_partials_packed(const double (&v)[W][VW], const PackLane& pl, double* partial) {
    __shared__ double sh[W * VW][kReduceThreads];
    const bool act = pl.roff < pl.rpb;
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
        for (int i = 0; i < VW; ++i) sh[w * VW + i][threadIdx.x] = act ? v[w][i] : 0.0;
    __syncthreads();
    const int nv = pl.nvp * VW;
    if (static_cast<int>(threadIdx.x) < nv) {
        const int pk = threadIdx.x / VW, i = threadIdx.x - pk * VW;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            double s = 0.0;
            for (int j = 0; j < pl.rpb; ++j) s += sh[w * VW + i][j * pl.nvp + pk];
            partial[(static_cast<int64_t>(blockIdx.x) * W + w) * nv + threadIdx.x] = s;
        }
    }
}

// Row/RHS position of this thread inside the reduction block layout.
struct RowLane {
    int rpb;   // rows per block step
    int roff;  // row offset of this thread (>= rpb: idle)
    int rhs;
};
__device__ __forceinline__ RowLane row_lane(int nv) {
    RowLane r;
    r.rpb = kReduceThreads / nv;
    r.roff = threadIdx.x / nv;
    r.rhs = threadIdx.x - r.roff * nv;
    return r;
}

// Per-block per-RHS partial sums of `width` doubles per thread.
template <int W>
__device__ __forceinline__ void block_partials(const double (&v)[W], int nv, const RowLane& rl, double* partial) {
    __shared__ double sh[W][kReduceThreads];
#pragma unroll
    for (int w = 0; w < W; ++w) sh[w][threadIdx.x] = (rl.roff < rl.rpb) ? v[w] : 0.0;
    __syncthreads();
    if (threadIdx.x < nv) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            double s = 0.0;
            for (int j = 0; j < rl.rpb; ++j) s += sh[w][j * nv + threadIdx.x];
            partial[(static_cast<int64_t>(blockIdx.x) * W + w) * nv + threadIdx.x] = s;
        }
    }
}

// out[rhs*W + w] = sum over blocks of partial[(b*W + w)*nv + rhs]; one block per (w, rhs).
// For W = 2 the result is interleaved (re, im) per RHS, i.e. usable as complex coefficients.
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partial, int64_t nblk, int width_w, int nv,
                                                  double* __restrict__ out) {
    __shared__ double sh[256];
    const int j = blockIdx.x;  // j = w*nv + rhs
    const int w = j / nv, rhs = j - w * nv;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += 256) s += partial[(b * width_w + w) * nv + rhs];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[rhs * width_w + w] = sh[0];
}

// out[b * nv + rhs] = sum of partial[i * nv + rhs] over i in [b * chunk, min((b + 1) * chunk, nblk)).  Thread t
// takes RHS t % nv and every (blockDim / nv)-th i of the range from t / nv on; lane 0 of each RHS then adds the
// lanes' sums in order.  blockDim is a multiple of nv.
constexpr int kRowSumBlocks = 256;
__global__ __launch_bounds__(256) void k_sum_ranges(const double* __restrict__ partial, int64_t nblk, int nv,
                                                    int64_t chunk, double* __restrict__ out) {
    __shared__ double sh[256];
    const int lanes = static_cast<int>(blockDim.x) / nv;
    const int t = threadIdx.x, rhs = t % nv, lane = t / nv;
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t i1 = i0 + chunk < nblk ? i0 + chunk : nblk;
    double s = 0.0;
    for (int64_t i = i0 + lane; i < i1; i += lanes) s += partial[i * nv + rhs];
    sh[t] = s;
    __syncthreads();
    if (lane == 0) {
        double a = 0.0;
        for (int l = 0; l < lanes; ++l) a += sh[l * nv + rhs];
        out[static_cast<int64_t>(blockIdx.x) * nv + rhs] = a;
    }
}

void finalize(const double* partial, int width_w, int nv, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(width_w * nv), dim3(256), 0, st, partial, static_cast<int64_t>(kReduceBlocks),
                       width_w, nv, out);
}

template <int VW, typename SX>
__global__ __launch_bounds__(kReduceThreads) void k_norm2(const SX* __restrict__ x, int64_t nrows, int nv,
                                                           double* __restrict__ partial) {
    const PackLane pl = pack_lane(nv / VW);
    double acc[1][VW] = {};
    if (pl.roff < pl.rpb) {
        const int64_t step = static_cast<int64_t>(gridDim.x) * pl.rpb;
#pragma unroll 2
        for (int64_t row = static_cast<int64_t>(blockIdx.x) * pl.rpb + pl.roff; row < nrows; row += step) {
            cx<double> v[VW];
            ldp<VW>(x + row * nv + pl.pk * VW, v);
#pragma unroll
            for (int i = 0; i < VW; ++i) acc[0][i] += v[i].re * v[i].re + v[i].im * v[i].im;
        }
    }
    block_partials_packed<1, VW>(acc, pl, partial);
}

template <int VW, typename SX, typename SY>
__global__ __launch_bounds__(kReduceThreads) void k_dot(const SX* __restrict__ x, const SY* __restrict__ y,
                                                         int64_t nrows, int nv, double* __restrict__ partial) {
    const PackLane pl = pack_lane(nv / VW);
    double acc[2][VW] = {};
    if (pl.roff < pl.rpb) {
        const int64_t step = static_cast<int64_t>(gridDim.x) * pl.rpb;
#pragma unroll 2
        for (int64_t row = static_cast<int64_t>(blockIdx.x) * pl.rpb + pl.roff; row < nrows; row += step) {
            cx<double> a[VW], b[VW];
            ldp<VW>(x + row * nv + pl.pk * VW, a);
            ldp<VW>(y + row * nv + pl.pk * VW, b);
#pragma unroll
            for (int i = 0; i < VW; ++i) {
                acc[0][i] += a[i].re * b[i].re + a[i].im * b[i].im;
                acc[1][i] += a[i].re * b[i].im - a[i].im * b[i].re;
            }
        }
    }
    block_partials_packed<2, VW>(acc, pl, partial);
}

// Elementwise kernels: grid-stride over complex elements, rhs = element % nv.
// Grid of an element-wise kernel: one element (or pack) per thread.  The kernels are grid-stride loops,
// so a capped grid is still correct; a grid covering every element measured 10-13 % faster than one of
// 8192 work-groups looping over it (FP32 x/p update at 32^3 x 64: 2.19 against 2.51 ms).
inline dim3 ew_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > (int64_t{1} << 30)) b = int64_t{1} << 30;
    if (b < 1) b = 1;
    return dim3(static_cast<unsigned>(b));
}

template <typename SX, typename SY>
__global__ __launch_bounds__(256) void k_caxpy(const SX* __restrict__ x, SY* __restrict__ y,
                                                const double2* __restrict__ a, int64_t n, int nv) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double2 al = a[i % nv];
        cx<double> yv = ldd(y + i);
        cfma(yv, cx<double>{al.x, al.y}, ldd(x + i));
        std_(y + i, yv);
    }
}

template <typename SX, typename SY>
__global__ __launch_bounds__(256) void k_cxpay(const SX* __restrict__ x, SY* __restrict__ y,
                                                const double2* __restrict__ a, int64_t n, int nv) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double2 al = a[i % nv];
        cx<double> v = ldd(x + i);
        cfma(v, cx<double>{al.x, al.y}, ldd(y + i));
        std_(y + i, v);
    }
}

template <typename SX, typename SY>
__global__ __launch_bounds__(256) void k_rscale(const SX* __restrict__ x, SY* __restrict__ y,
                                                 const double* __restrict__ s, int64_t n, int nv) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        std_(y + i, cscale(s[i % nv], ldd(x + i)));
}

template <typename SX, typename SY>
__global__ __launch_bounds__(256) void k_cast(const SX* __restrict__ x, SY* __restrict__ y, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        std_(y + i, ldd(x + i));
}

// float -> bf16 directly (single rounding) for the FP32 -> BF16 cast.
__global__ __launch_bounds__(256) void k_cast_f2b(const float2* __restrict__ x, bf16x2* __restrict__ y, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        io<float, bf16x2>::st(y + i, io<float, float2>::ld(x + i));
}

template <typename SB, typename SY>
__global__ __launch_bounds__(256) void k_bminus(const SB* __restrict__ b, SY* __restrict__ y, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        std_(y + i, csub(ldd(b + i), ldd(y + i)));
}

template <typename SB, typename SQ, typename SR>
__global__ __launch_bounds__(256) void k_sub(const SB* __restrict__ b, const SQ* __restrict__ q, SR* __restrict__ r,
                                              int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        std_(r + i, csub(ldd(b + i), ldd(q + i)));
}

// gamma_5 = diag(1,1,-1,-1) on [site][colour][spin][rhs]
template <typename S>
__global__ __launch_bounds__(256) void k_gamma5(const S* __restrict__ x, S* __restrict__ y, int64_t n, int nv) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int spin = static_cast<int>((i / nv) & 3);
        cx<double> v = ldd(x + i);
        std_(y + i, spin < 2 ? v : cscale(-1.0, v));
    }
}

// epsilon = (-1)^(x+y+z+t) on [site][colour][rhs]
template <typename S>
__global__ __launch_bounds__(256) void k_epsilon(const S* __restrict__ x, S* __restrict__ y, int64_t n, int per_site,
                                                 Geom g) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const Coord c = site_coord(i / per_site, g);
        cx<double> v = ldd(x + i);
        std_(y + i, ((c.x + c.y + c.z + c.t) & 1) ? cscale(-1.0, v) : v);
    }
}

// r -= alpha q ; partial ||r||^2
template <int VW, typename SR, typename SQ>
__global__ __launch_bounds__(kReduceThreads) void k_r_update(SR* __restrict__ r, const SQ* __restrict__ q,
                                                              const double2* __restrict__ alpha, int64_t nrows,
                                                              int nv, double* __restrict__ partial) {
    const PackLane pl = pack_lane(nv / VW);
    double acc[1][VW] = {};
    if (pl.roff < pl.rpb) {
        cx<double> ma[VW];
#pragma unroll
        for (int i = 0; i < VW; ++i) {
            const double2 al = alpha[pl.pk * VW + i];
            ma[i] = {-al.x, -al.y};
        }
        const int64_t step = static_cast<int64_t>(gridDim.x) * pl.rpb;
#pragma unroll 2
        for (int64_t row = static_cast<int64_t>(blockIdx.x) * pl.rpb + pl.roff; row < nrows; row += step) {
            const int64_t e = row * nv + pl.pk * VW;
            cx<double> rv[VW], qv[VW];
            ldp<VW>(r + e, rv);
            ldp<VW>(q + e, qv);
#pragma unroll
            for (int i = 0; i < VW; ++i) cfma(rv[i], ma[i], qv[i]);
            stp<VW>(r + e, rv);
#pragma unroll
            for (int i = 0; i < VW; ++i) {
                const cx<double> st = stored_value<SR>(rv[i]);  // norm of the value as stored
                acc[0][i] += st.re * st.re + st.im * st.im;
            }
        }
    }
    block_partials_packed<1, VW>(acc, pl, partial);
}

// x += alpha p ; p = r + beta p (packs of VW elements, grid-stride)
template <int VW, typename SX, typename SP, typename SR>
__global__ __launch_bounds__(256) void k_xp_update(SX* __restrict__ x, SP* __restrict__ p, const SR* __restrict__ r,
                                                    const double2* __restrict__ alpha,
                                                    const double2* __restrict__ beta, int64_t n, int nv) {
    const int64_t npk = n / VW;
    const int nvp = nv / VW;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < npk;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int k0 = static_cast<int>(i % nvp) * VW;
        const int64_t e = i * VW;
        cx<double> pv[VW], xv[VW], rv[VW];
        ldp<VW>(p + e, pv);
        ldp<VW>(x + e, xv);
        ldp<VW>(r + e, rv);
#pragma unroll
        for (int j = 0; j < VW; ++j) {
            const double2 al = alpha[k0 + j], be = beta[k0 + j];
            cfma(xv[j], cx<double>{al.x, al.y}, pv[j]);
            cfma(rv[j], cx<double>{be.x, be.y}, pv[j]);
        }
        stp<VW>(x + e, xv);
        stp<VW>(p + e, rv);
    }
}

// x += alpha p ; p = r + beta p ; partial <r, p> of the new p as stored (the line-search numerator
// of the next step; reads and writes nothing beyond k_xp_update)
template <int VW, typename SX, typename SP, typename SR>
__global__ __launch_bounds__(kReduceThreads) void k_xp_update_dot(SX* __restrict__ x, SP* __restrict__ p,
                                                                   const SR* __restrict__ r,
                                                                   const double2* __restrict__ alpha,
                                                                   const double2* __restrict__ beta, int64_t nrows,
                                                                   int nv, double* __restrict__ partial) {
    const PackLane pl = pack_lane(nv / VW);
    double acc[2][VW] = {};
    if (pl.roff < pl.rpb) {
        cx<double> al[VW], be[VW];
#pragma unroll
        for (int i = 0; i < VW; ++i) {
            const double2 a = alpha[pl.pk * VW + i], b = beta[pl.pk * VW + i];
            al[i] = {a.x, a.y};
            be[i] = {b.x, b.y};
        }
        const int64_t step = static_cast<int64_t>(gridDim.x) * pl.rpb;
#pragma unroll 2
        for (int64_t row = static_cast<int64_t>(blockIdx.x) * pl.rpb + pl.roff; row < nrows; row += step) {
            const int64_t e = row * nv + pl.pk * VW;
            cx<double> pv[VW], xv[VW], rv[VW], np[VW];
            ldp<VW>(p + e, pv);
            ldp<VW>(x + e, xv);
            ldp<VW>(r + e, rv);
#pragma unroll
            for (int i = 0; i < VW; ++i) {
                cfma(xv[i], al[i], pv[i]);
                np[i] = rv[i];
                cfma(np[i], be[i], pv[i]);
            }
            stp<VW>(x + e, xv);
            stp<VW>(p + e, np);
#pragma unroll
            for (int i = 0; i < VW; ++i) {
                const cx<double> ps = stored_value<SP>(np[i]);  // <r, p> of p as stored
                acc[0][i] += rv[i].re * ps.re + rv[i].im * ps.im;
                acc[1][i] += rv[i].re * ps.im - rv[i].im * ps.re;
            }
        }
    }
    block_partials_packed<2, VW>(acc, pl, partial);
}

// The same update with kBurstRows rows per thread, taken once with every load issued before any
// arithmetic (element-wise kernels whose threads loop over many rows measured 10-13 % slower); one
// partial per block, kBurstRows * rows-per-block rows per block.
constexpr int kBurstRows = 4;
template <int VW, typename SX, typename SP, typename SR>
__global__ __launch_bounds__(kReduceThreads) void k_xp_update_dot_burst(SX* __restrict__ x, SP* __restrict__ p,
                                                                         const SR* __restrict__ r,
                                                                         const double2* __restrict__ alpha,
                                                                         const double2* __restrict__ beta,
                                                                         int64_t nrows, int nv,
                                                                         double* __restrict__ partial) {
    const PackLane pl = pack_lane(nv / VW);
    double acc[2][VW] = {};
    if (pl.roff < pl.rpb) {
        cx<double> al[VW], be[VW];
#pragma unroll
        for (int i = 0; i < VW; ++i) {
            const double2 a = alpha[pl.pk * VW + i], b = beta[pl.pk * VW + i];
            al[i] = {a.x, a.y};
            be[i] = {b.x, b.y};
        }
        const int64_t row0 = static_cast<int64_t>(blockIdx.x) * (kBurstRows * pl.rpb) + pl.roff;
        cx<double> pv[kBurstRows][VW], xv[kBurstRows][VW], rv[kBurstRows][VW];
#pragma unroll
        for (int q = 0; q < kBurstRows; ++q) {
            const int64_t row = row0 + static_cast<int64_t>(q) * pl.rpb;
            if (row < nrows) {
                const int64_t e = row * nv + pl.pk * VW;
                ldp<VW>(p + e, pv[q]);
                ldp<VW>(x + e, xv[q]);
                ldp<VW>(r + e, rv[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < kBurstRows; ++q) {
            const int64_t row = row0 + static_cast<int64_t>(q) * pl.rpb;
            if (row >= nrows) continue;
            const int64_t e = row * nv + pl.pk * VW;
            cx<double> np[VW];
#pragma unroll
            for (int i = 0; i < VW; ++i) {
                cfma(xv[q][i], al[i], pv[q][i]);
                np[i] = rv[q][i];
                cfma(np[i], be[i], pv[q][i]);
            }
            stp<VW>(x + e, xv[q]);
            stp<VW>(p + e, np);
#pragma unroll
            for (int i = 0; i < VW; ++i) {
                const cx<double> ps = stored_value<SP>(np[i]);  // <r, p> of p as stored
                acc[0][i] += rv[q][i].re * ps.re + rv[q][i].im * ps.im;
                acc[1][i] += rv[q][i].re * ps.im - rv[q][i].im * ps.re;
            }
        }
    }
    block_partials_packed<2, VW>(acc, pl, partial);
}

inline int64_t burst_blocks(int64_t nrows, int nv, int vw) {
    const int64_t rows_per_block = static_cast<int64_t>(kBurstRows) * (kReduceThreads / (nv / vw));
    return (nrows + rows_per_block - 1) / rows_per_block;
}

// BiCGstab: x += alpha p + omega s ; r = s - omega t ; partial ||r||^2
template <typename S>
__global__ __launch_bounds__(kReduceThreads) void k_bicg_xr(S* __restrict__ x, const S* __restrict__ p,
                                                             const S* __restrict__ s, const S* __restrict__ t,
                                                             S* __restrict__ r, const double2* __restrict__ alpha,
                                                             const double2* __restrict__ omega, int64_t nrows, int nv,
                                                             double* __restrict__ partial) {
    const RowLane rl = row_lane(nv);
    double acc[1] = {0.0};
    if (rl.roff < rl.rpb) {
        const double2 al = alpha[rl.rhs], om = omega[rl.rhs];
        const cx<double> a{al.x, al.y}, w{om.x, om.y}, mw{-om.x, -om.y};
        const int64_t step = static_cast<int64_t>(gridDim.x) * rl.rpb;
#pragma unroll 4
        for (int64_t row = static_cast<int64_t>(blockIdx.x) * rl.rpb + rl.roff; row < nrows; row += step) {
            const int64_t i = row * nv + rl.rhs;
            const cx<double> sv = ldd(s + i);
            cx<double> xv = ldd(x + i);
            cfma(xv, a, ldd(p + i));
            cfma(xv, w, sv);
            std_(x + i, xv);
            cx<double> rv = sv;
            cfma(rv, mw, ldd(t + i));
            std_(r + i, rv);
            const cx<double> st = stored_value<S>(rv);
            acc[0] += st.re * st.re + st.im * st.im;
        }
    }
    block_partials<1>(acc, nv, rl, partial);
}

// BiCGstab: p = r + beta (p - omega v)
template <typename S>
__global__ __launch_bounds__(256) void k_bicg_p(S* __restrict__ p, const S* __restrict__ r, const S* __restrict__ v,
                                                 const double2* __restrict__ beta, const double2* __restrict__ omega,
                                                 int64_t n, int nv) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int k = static_cast<int>(i % nv);
        const double2 be = beta[k], om = omega[k];
        cx<double> t = ldd(p + i);
        cfma(t, cx<double>{-om.x, -om.y}, ldd(v + i));
        cx<double> o = ldd(r + i);
        cfma(o, cx<double>{be.x, be.y}, t);
        std_(p + i, o);
    }
}

// BiCGstab: s = r - alpha v
template <typename S>
__global__ __launch_bounds__(256) void k_bicg_s(S* __restrict__ s, const S* __restrict__ r, const S* __restrict__ v,
                                                 const double2* __restrict__ alpha, int64_t n, int nv) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double2 al = alpha[i % nv];
        cx<double> o = ldd(r + i);
        cfma(o, cx<double>{-al.x, -al.y}, ldd(v + i));
        std_(s + i, o);
    }
}

}  // namespace

void finalize_blocks(const double* partial, int64_t nblk, int nv, double* scratch, double* out, hipStream_t st) {
    // stage 1: kRowSumBlocks blocks each add a contiguous range of blocks' partials for every RHS (coalesced
    // reads); stage 2 adds the kRowSumBlocks results per RHS.  Both orders are fixed.
    const int lanes = 256 / nv;
    const int64_t chunk = (nblk + kRowSumBlocks - 1) / kRowSumBlocks;
    hipLaunchKernelGGL(k_sum_ranges, dim3(kRowSumBlocks), dim3(lanes * nv), 0, st, partial, nblk, nv, chunk, scratch);
    hipLaunchKernelGGL(k_finalize, dim3(nv), dim3(256), 0, st, scratch, static_cast<int64_t>(kRowSumBlocks), 1, nv,
                       out);
}

int blas_norm2(dirac_prec p, const void* x, int64_t nrows, int nv, double* partial, double* out, hipStream_t st) {
    return with_prec(p, [&](auto tx) {
        using SX = typename decltype(tx)::type;
        constexpr int VW = pack_width<SX>();
        if (pack_ok(VW, nv, {x}))
            hipLaunchKernelGGL((k_norm2<VW, SX>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, st,
                               static_cast<const SX*>(x), nrows, nv, partial);
        else
            hipLaunchKernelGGL((k_norm2<1, SX>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, st,
                               static_cast<const SX*>(x), nrows, nv, partial);
        finalize(partial, 1, nv, out, st);
        return DIRAC_OK;
    });
}

int blas_dot(dirac_prec px, const void* x, dirac_prec py, const void* y, int64_t nrows, int nv, double* partial,
             double* out, hipStream_t st) {
    return with_prec(px, [&](auto tx) {
        return with_prec(py, [&](auto ty) {
            using SX = typename decltype(tx)::type;
            using SY = typename decltype(ty)::type;
            constexpr int VW = pack_width<SX, SY>();
            if (pack_ok(VW, nv, {x, y}))
                hipLaunchKernelGGL((k_dot<VW, SX, SY>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, st,
                                   static_cast<const SX*>(x), static_cast<const SY*>(y), nrows, nv, partial);
            else
                hipLaunchKernelGGL((k_dot<1, SX, SY>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, st,
                                   static_cast<const SX*>(x), static_cast<const SY*>(y), nrows, nv, partial);
            finalize(partial, 2, nv, out, st);
            return DIRAC_OK;
        });
    });
}

int blas_caxpy(dirac_prec px, const void* x, dirac_prec py, void* y, const double* a, int64_t nrows, int nv,
               hipStream_t st) {
    const int64_t n = nrows * nv;
    return with_prec(px, [&](auto tx) {
        return with_prec(py, [&](auto ty) {
            using SX = typename decltype(tx)::type;
            using SY = typename decltype(ty)::type;
            hipLaunchKernelGGL((k_caxpy<SX, SY>), ew_grid(n), dim3(256), 0, st, static_cast<const SX*>(x),
                               static_cast<SY*>(y), reinterpret_cast<const double2*>(a), n, nv);
            return DIRAC_OK;
        });
    });
}

int blas_cxpay(dirac_prec px, const void* x, dirac_prec py, void* y, const double* a, int64_t nrows, int nv,
               hipStream_t st) {
    const int64_t n = nrows * nv;
    return with_prec(px, [&](auto tx) {
        return with_prec(py, [&](auto ty) {
            using SX = typename decltype(tx)::type;
            using SY = typename decltype(ty)::type;
            hipLaunchKernelGGL((k_cxpay<SX, SY>), ew_grid(n), dim3(256), 0, st, static_cast<const SX*>(x),
                               static_cast<SY*>(y), reinterpret_cast<const double2*>(a), n, nv);
            return DIRAC_OK;
        });
    });
}

int blas_rscale(dirac_prec px, const void* x, dirac_prec py, void* y, const double* s, int64_t nrows, int nv,
                hipStream_t st) {
    const int64_t n = nrows * nv;
    return with_prec(px, [&](auto tx) {
        return with_prec(py, [&](auto ty) {
            using SX = typename decltype(tx)::type;
            using SY = typename decltype(ty)::type;
            hipLaunchKernelGGL((k_rscale<SX, SY>), ew_grid(n), dim3(256), 0, st, static_cast<const SX*>(x),
                               static_cast<SY*>(y), s, n, nv);
            return DIRAC_OK;
        });
    });
}

int blas_cast(dirac_prec px, const void* x, dirac_prec py, void* y, int64_t n, hipStream_t st) {
    if (px == DIRAC_FP32 && py == DIRAC_BF16) {
        hipLaunchKernelGGL(k_cast_f2b, ew_grid(n), dim3(256), 0, st, static_cast<const float2*>(x),
                           static_cast<bf16x2*>(y), n);
        return DIRAC_OK;
    }
    return with_prec(px, [&](auto tx) {
        return with_prec(py, [&](auto ty) {
            using SX = typename decltype(tx)::type;
            using SY = typename decltype(ty)::type;
            hipLaunchKernelGGL((k_cast<SX, SY>), ew_grid(n), dim3(256), 0, st, static_cast<const SX*>(x),
                               static_cast<SY*>(y), n);
            return DIRAC_OK;
        });
    });
}

int blas_bminus(dirac_prec pb, const void* b, dirac_prec py, void* y, int64_t nrows, int nv, hipStream_t st) {
    const int64_t n = nrows * nv;
    return with_prec(pb, [&](auto tb) {
        return with_prec(py, [&](auto ty) {
            using SB = typename decltype(tb)::type;
            using SY = typename decltype(ty)::type;
            hipLaunchKernelGGL((k_bminus<SB, SY>), ew_grid(n), dim3(256), 0, st, static_cast<const SB*>(b),
                               static_cast<SY*>(y), n);
            return DIRAC_OK;
        });
    });
}

int blas_sub(dirac_prec pb, const void* b, dirac_prec pq, const void* q, dirac_prec pr, void* r, int64_t n,
             hipStream_t st) {
    return with_prec(pb, [&](auto tb) {
        return with_prec(pq, [&](auto tq) {
            return with_prec(pr, [&](auto tr) {
                using SB = typename decltype(tb)::type;
                using SQ = typename decltype(tq)::type;
                using SR = typename decltype(tr)::type;
                hipLaunchKernelGGL((k_sub<SB, SQ, SR>), ew_grid(n), dim3(256), 0, st, static_cast<const SB*>(b),
                                   static_cast<const SQ*>(q), static_cast<SR*>(r), n);
                return DIRAC_OK;
            });
        });
    });
}

int blas_gamma5(dirac_op op, dirac_prec p, const void* x, void* y, int nc, int nv, const Geom& g, hipStream_t st) {
    return with_prec(p, [&](auto tx) {
        using S = typename decltype(tx)::type;
        if (op == DIRAC_STAGGERED) {
            const int64_t n = g.vol * nc * nv;
            hipLaunchKernelGGL((k_epsilon<S>), ew_grid(n), dim3(256), 0, st, static_cast<const S*>(x),
                               static_cast<S*>(y), n, nc * nv, g);
        } else {
            const int64_t n = g.vol * nc * 4 * nv;
            hipLaunchKernelGGL((k_gamma5<S>), ew_grid(n), dim3(256), 0, st, static_cast<const S*>(x),
                               static_cast<S*>(y), n, nv);
        }
        return DIRAC_OK;
    });
}

int fused_r_update(dirac_prec pr, void* r, dirac_prec pq, const void* q, const double* alpha, int64_t nrows, int nv,
                   double* partial, double* rr, hipStream_t st) {
    return with_prec(pr, [&](auto tr) {
        return with_prec(pq, [&](auto tq) {
            using SR = typename decltype(tr)::type;
            using SQ = typename decltype(tq)::type;
            constexpr int VW = pack_width<SR, SQ>();
            if (pack_ok(VW, nv, {r, q}))
                hipLaunchKernelGGL((k_r_update<VW, SR, SQ>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, st,
                                   static_cast<SR*>(r), static_cast<const SQ*>(q),
                                   reinterpret_cast<const double2*>(alpha), nrows, nv, partial);
            else
                hipLaunchKernelGGL((k_r_update<1, SR, SQ>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, st,
                                   static_cast<SR*>(r), static_cast<const SQ*>(q),
                                   reinterpret_cast<const double2*>(alpha), nrows, nv, partial);
            finalize(partial, 1, nv, rr, st);
            return DIRAC_OK;
        });
    });
}

int fused_xp_update(dirac_prec px, void* x, dirac_prec pp, void* p, dirac_prec prr, const void* r, const double* alpha,
                    const double* beta, int64_t nrows, int nv, hipStream_t st) {
    const int64_t n = nrows * nv;
    return with_prec(px, [&](auto tx) {
        return with_prec(pp, [&](auto tp) {
            return with_prec(prr, [&](auto trr) {
                using SX = typename decltype(tx)::type;
                using SP = typename decltype(tp)::type;
                using SR = typename decltype(trr)::type;
                constexpr int VW = pack_width<SX, SP, SR>();
                if (pack_ok(VW, nv, {x, p, r}))
                    hipLaunchKernelGGL((k_xp_update<VW, SX, SP, SR>), ew_grid(n / VW), dim3(256), 0, st,
                                       static_cast<SX*>(x), static_cast<SP*>(p), static_cast<const SR*>(r),
                                       reinterpret_cast<const double2*>(alpha), reinterpret_cast<const double2*>(beta),
                                       n, nv);
                else
                    hipLaunchKernelGGL((k_xp_update<1, SX, SP, SR>), ew_grid(n), dim3(256), 0, st,
                                       static_cast<SX*>(x), static_cast<SP*>(p), static_cast<const SR*>(r),
                                       reinterpret_cast<const double2*>(alpha), reinterpret_cast<const double2*>(beta),
                                       n, nv);
                return DIRAC_OK;
            });
        });
    });
}

size_t burst_partial_doubles(int64_t nrows, int nv) {
    // the largest block count is that of single-column packs; 2 nv columns must fit one row-sum block
    if (nv < 1 || 2 * nv > 256) return 0;
    return static_cast<size_t>(burst_blocks(nrows, nv, 1)) * 2 * nv;
}

int fused_xp_update_dot(dirac_prec px, void* x, dirac_prec pp, void* p, dirac_prec prr, const void* r,
                        const double* alpha, const double* beta, int64_t nrows, int nv, double* partial, double* rp,
                        hipStream_t st, double* burst, size_t burst_doubles) {
    return with_prec(px, [&](auto tx) {
        return with_prec(pp, [&](auto tp) {
            return with_prec(prr, [&](auto trr) {
                using SX = typename decltype(tx)::type;
                using SP = typename decltype(tp)::type;
                using SR = typename decltype(trr)::type;
                constexpr int VW = pack_width<SX, SP, SR>();
                const int vw = pack_ok(VW, nv, {x, p, r}) ? VW : 1;
                const int64_t nb = burst_blocks(nrows, nv, vw);
                if (burst && 2 * nv <= 256 && static_cast<size_t>(nb) * 2 * nv <= burst_doubles) {
                    if (vw == VW)
                        hipLaunchKernelGGL((k_xp_update_dot_burst<VW, SX, SP, SR>), dim3(static_cast<unsigned>(nb)),
                                           dim3(kReduceThreads), 0, st, static_cast<SX*>(x), static_cast<SP*>(p),
                                           static_cast<const SR*>(r), reinterpret_cast<const double2*>(alpha),
                                           reinterpret_cast<const double2*>(beta), nrows, nv, burst);
                    else
                        hipLaunchKernelGGL((k_xp_update_dot_burst<1, SX, SP, SR>), dim3(static_cast<unsigned>(nb)),
                                           dim3(kReduceThreads), 0, st, static_cast<SX*>(x), static_cast<SP*>(p),
                                           static_cast<const SR*>(r), reinterpret_cast<const double2*>(alpha),
                                           reinterpret_cast<const double2*>(beta), nrows, nv, burst);
                    // the partials are [block][w][rhs]: rows of 2 nv columns summed in ranges, then per (rhs, w)
                    const int lanes = 256 / (2 * nv);
                    const int64_t chunk = (nb + kRowSumBlocks - 1) / kRowSumBlocks;
                    hipLaunchKernelGGL(k_sum_ranges, dim3(kRowSumBlocks), dim3(lanes * 2 * nv), 0, st, burst, nb, 2 * nv,
                                       chunk, partial);
                    hipLaunchKernelGGL(k_finalize, dim3(2 * nv), dim3(256), 0, st, partial,
                                       static_cast<int64_t>(kRowSumBlocks), 2, nv, rp);
                    return DIRAC_OK;
                }
                if (vw == VW)
                    hipLaunchKernelGGL((k_xp_update_dot<VW, SX, SP, SR>), dim3(kReduceBlocks), dim3(kReduceThreads), 0,
                                       st, static_cast<SX*>(x), static_cast<SP*>(p), static_cast<const SR*>(r),
                                       reinterpret_cast<const double2*>(alpha), reinterpret_cast<const double2*>(beta),
                                       nrows, nv, partial);
                else
                    hipLaunchKernelGGL((k_xp_update_dot<1, SX, SP, SR>), dim3(kReduceBlocks), dim3(kReduceThreads), 0,
                                       st, static_cast<SX*>(x), static_cast<SP*>(p), static_cast<const SR*>(r),
                                       reinterpret_cast<const double2*>(alpha), reinterpret_cast<const double2*>(beta),
                                       nrows, nv, partial);
                finalize(partial, 2, nv, rp, st);
                return DIRAC_OK;
            });
        });
    });
}

// ---------------------------------------------------------------------------
// Reduction partials without a workspace argument, for callers that cannot allocate: a file-scope
// device array sized for the largest N_v (each device holds its own copy for the life of the process).
// Host code reaches it only through the address hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchDoubles = static_cast<size_t>(kReduceBlocks) * 2 * 256;  // 8 MiB
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

size_t static_scratch_doubles() { return kScratchDoubles; }

int static_scratch(double** out) {
    int dev = 0;
    DIRAC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DIRAC_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        DIRAC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return DIRAC_OK;
}

int fused_bicg_xr(dirac_prec p, void* x, const void* pv, const void* s, const void* t, void* r, const double* alpha,
                  const double* omega, int64_t nrows, int nv, double* partial, double* rr, hipStream_t st) {
    return with_prec(p, [&](auto tp) {
        using S = typename decltype(tp)::type;
        hipLaunchKernelGGL((k_bicg_xr<S>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, st, static_cast<S*>(x),
                           static_cast<const S*>(pv), static_cast<const S*>(s), static_cast<const S*>(t),
                           static_cast<S*>(r), reinterpret_cast<const double2*>(alpha),
                           reinterpret_cast<const double2*>(omega), nrows, nv, partial);
        finalize(partial, 1, nv, rr, st);
        return DIRAC_OK;
    });
}

int fused_bicg_p(dirac_prec p, void* pv, const void* r, const void* v, const double* beta, const double* omega,
                 int64_t nrows, int nv, hipStream_t st) {
    const int64_t n = nrows * nv;
    return with_prec(p, [&](auto tp) {
        using S = typename decltype(tp)::type;
        hipLaunchKernelGGL((k_bicg_p<S>), ew_grid(n), dim3(256), 0, st, static_cast<S*>(pv), static_cast<const S*>(r),
                           static_cast<const S*>(v), reinterpret_cast<const double2*>(beta),
                           reinterpret_cast<const double2*>(omega), n, nv);
        return DIRAC_OK;
    });
}

int fused_bicg_s(dirac_prec p, void* s, const void* r, const void* v, const double* alpha, int64_t nrows, int nv,
                 hipStream_t st) {
    const int64_t n = nrows * nv;
    return with_prec(p, [&](auto tp) {
        using S = typename decltype(tp)::type;
        hipLaunchKernelGGL((k_bicg_s<S>), ew_grid(n), dim3(256), 0, st, static_cast<S*>(s), static_cast<const S*>(r),
                           static_cast<const S*>(v), reinterpret_cast<const double2*>(alpha), n, nv);
        return DIRAC_OK;
    });
}

}  // namespace dirac
