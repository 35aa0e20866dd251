// Multi-RHS BLAS-1 and the fused Krylov update kernels (Sec. 3: norms, dot products,
// "incr"/"anti" multiply-adds, casts, gamma_5 / epsilon).
//
// A vector is `nrows` rows of `nv` complex numbers (the right-hand-side index is fastest).
// Arithmetic is FP64 whatever the storage precision, and so is every accumulation.
// Reductions are two-pass and deterministic: a fixed grid of kReduceBlocks blocks, each
// block handles rows blockIdx + k * gridDim in a fixed order and reduces per RHS through
// LDS in a fixed order, then one block per output value adds the block partials with a
// fixed tree.  Repeated runs give bitwise identical results.
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
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partial, int nblk, int width_w, int nv,
                                                  double* __restrict__ out) {
    __shared__ double sh[256];
    const int j = blockIdx.x;  // j = w*nv + rhs
    const int w = j / nv, rhs = j - w * nv;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += partial[(static_cast<int64_t>(b) * width_w + w) * nv + rhs];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[rhs * width_w + w] = sh[0];
}

void finalize(const double* partial, int width_w, int nv, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(width_w * nv), dim3(256), 0, st, partial, kReduceBlocks, width_w, nv, out);
}

template <typename SX>
__global__ __launch_bounds__(kReduceThreads) void k_norm2(const SX* __restrict__ x, int64_t nrows, int nv,
                                                           double* __restrict__ partial) {
    const RowLane rl = row_lane(nv);
    double acc[1] = {0.0};
    if (rl.roff < rl.rpb) {
        const int64_t step = static_cast<int64_t>(gridDim.x) * rl.rpb;
#pragma unroll 4
        for (int64_t row = static_cast<int64_t>(blockIdx.x) * rl.rpb + rl.roff; row < nrows; row += step) {
            cx<double> v = ldd(x + row * nv + rl.rhs);
            acc[0] += v.re * v.re + v.im * v.im;
        }
    }
    block_partials<1>(acc, nv, rl, partial);
}

template <typename SX, typename SY>
__global__ __launch_bounds__(kReduceThreads) void k_dot(const SX* __restrict__ x, const SY* __restrict__ y,
                                                         int64_t nrows, int nv, double* __restrict__ partial) {
    const RowLane rl = row_lane(nv);
    double acc[2] = {0.0, 0.0};
    if (rl.roff < rl.rpb) {
        const int64_t step = static_cast<int64_t>(gridDim.x) * rl.rpb;
#pragma unroll 4
        for (int64_t row = static_cast<int64_t>(blockIdx.x) * rl.rpb + rl.roff; row < nrows; row += step) {
            cx<double> a = ldd(x + row * nv + rl.rhs);
            cx<double> b = ldd(y + row * nv + rl.rhs);
            acc[0] += a.re * b.re + a.im * b.im;
            acc[1] += a.re * b.im - a.im * b.re;
        }
    }
    block_partials<2>(acc, nv, rl, partial);
}

// Elementwise kernels: grid-stride over complex elements, rhs = element % nv.
inline dim3 ew_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 256 * 32) b = 256 * 32;
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
template <typename SR, typename SQ>
__global__ __launch_bounds__(kReduceThreads) void k_r_update(SR* __restrict__ r, const SQ* __restrict__ q,
                                                              const double2* __restrict__ alpha, int64_t nrows,
                                                              int nv, double* __restrict__ partial) {
    const RowLane rl = row_lane(nv);
    double acc[1] = {0.0};
    if (rl.roff < rl.rpb) {
        const double2 al = alpha[rl.rhs];
        const cx<double> ma{-al.x, -al.y};
        const int64_t step = static_cast<int64_t>(gridDim.x) * rl.rpb;
#pragma unroll 4
        for (int64_t row = static_cast<int64_t>(blockIdx.x) * rl.rpb + rl.roff; row < nrows; row += step) {
            const int64_t i = row * nv + rl.rhs;
            cx<double> rv = ldd(r + i);
            cfma(rv, ma, ldd(q + i));
            std_(r + i, rv);
            const cx<double> st = stored_value<SR>(rv);  // norm of the value as stored
            acc[0] += st.re * st.re + st.im * st.im;
        }
    }
    block_partials<1>(acc, nv, rl, partial);
}

// x += alpha p ; p = r + beta p
template <typename SX, typename SP, typename SR>
__global__ __launch_bounds__(256) void k_xp_update(SX* __restrict__ x, SP* __restrict__ p, const SR* __restrict__ r,
                                                    const double2* __restrict__ alpha,
                                                    const double2* __restrict__ beta, int64_t n, int nv) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int k = static_cast<int>(i % nv);
        const double2 al = alpha[k], be = beta[k];
        const cx<double> pv = ldd(p + i);
        cx<double> xv = ldd(x + i);
        cfma(xv, cx<double>{al.x, al.y}, pv);
        std_(x + i, xv);
        cx<double> np = ldd(r + i);
        cfma(np, cx<double>{be.x, be.y}, pv);
        std_(p + i, np);
    }
}

// x += alpha p ; p = r + beta p ; partial <r, p> of the new p as stored (the line-search numerator
// of the next step; reads and writes nothing beyond k_xp_update)
template <typename SX, typename SP, typename SR>
__global__ __launch_bounds__(kReduceThreads) void k_xp_update_dot(SX* __restrict__ x, SP* __restrict__ p,
                                                                   const SR* __restrict__ r,
                                                                   const double2* __restrict__ alpha,
                                                                   const double2* __restrict__ beta, int64_t nrows,
                                                                   int nv, double* __restrict__ partial) {
    const RowLane rl = row_lane(nv);
    double acc[2] = {0.0, 0.0};
    if (rl.roff < rl.rpb) {
        const double2 al = alpha[rl.rhs], be = beta[rl.rhs];
        const int64_t step = static_cast<int64_t>(gridDim.x) * rl.rpb;
#pragma unroll 4
        for (int64_t row = static_cast<int64_t>(blockIdx.x) * rl.rpb + rl.roff; row < nrows; row += step) {
            const int64_t i = row * nv + rl.rhs;
            const cx<double> pv = ldd(p + i);
            cx<double> xv = ldd(x + i);
            cfma(xv, cx<double>{al.x, al.y}, pv);
            std_(x + i, xv);
            const cx<double> rv = ldd(r + i);
            cx<double> np = rv;
            cfma(np, cx<double>{be.x, be.y}, pv);
            std_(p + i, np);
            const cx<double> ps = stored_value<SP>(np);  // <r, p> of p as stored
            acc[0] += rv.re * ps.re + rv.im * ps.im;
            acc[1] += rv.re * ps.im - rv.im * ps.re;
        }
    }
    block_partials<2>(acc, nv, rl, partial);
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

int blas_norm2(dirac_prec p, const void* x, int64_t nrows, int nv, double* partial, double* out, hipStream_t st) {
    return with_prec(p, [&](auto tx) {
        using SX = typename decltype(tx)::type;
        hipLaunchKernelGGL((k_norm2<SX>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, st,
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
            hipLaunchKernelGGL((k_dot<SX, SY>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, st,
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
            hipLaunchKernelGGL((k_r_update<SR, SQ>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, st,
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
                hipLaunchKernelGGL((k_xp_update<SX, SP, SR>), ew_grid(n), dim3(256), 0, st, static_cast<SX*>(x),
                                   static_cast<SP*>(p), static_cast<const SR*>(r),
                                   reinterpret_cast<const double2*>(alpha), reinterpret_cast<const double2*>(beta), n,
                                   nv);
                return DIRAC_OK;
            });
        });
    });
}

int fused_xp_update_dot(dirac_prec px, void* x, dirac_prec pp, void* p, dirac_prec prr, const void* r,
                        const double* alpha, const double* beta, int64_t nrows, int nv, double* partial, double* rp,
                        hipStream_t st) {
    return with_prec(px, [&](auto tx) {
        return with_prec(pp, [&](auto tp) {
            return with_prec(prr, [&](auto trr) {
                using SX = typename decltype(tx)::type;
                using SP = typename decltype(tp)::type;
                using SR = typename decltype(trr)::type;
                hipLaunchKernelGGL((k_xp_update_dot<SX, SP, SR>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, st,
                                   static_cast<SX*>(x), static_cast<SP*>(p), static_cast<const SR*>(r),
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
