// Wilson Dirac operator D_W and its adjoint (Sec. 5, Eq. app_wils; r = 1, c_SW = 0).
//
//   (D_W u)(n)   = (4+m) u(n) - 1/2 sum_mu [(1 - g_mu) U_mu(n) u(n+mu) + (1 + g_mu) U_mu(n-mu)^+ u(n-mu)]
//   (D_W^+ u)(n) = (4+m) u(n) - 1/2 sum_mu [(1 + g_mu) U_mu(n) u(n+mu) + (1 - g_mu) U_mu(n-mu)^+ u(n-mu)]
//
// Each hop uses the spin-projection trick of App. A: (1 +- g_mu) has rank two, so the
// neighbour spinor is first reduced to two spin components h0, h1 (chiral basis), only
// those are multiplied by the Nc x Nc link, and the other two rows are rebuilt from them.
// One thread owns one site and RB consecutive right-hand sides; every output element is
// written once (no atomics).  Fermion fields pick up -1 on t-wrapping hops when
// antiperiodic in t.
#include "common.h"
#include "kernels.h"

namespace dirac {

namespace {

// Half spinor of (1 + SIG g_MU) psi in the chiral basis: rows 0 and 1.
template <int MU, int SIG, typename R>
__device__ __forceinline__ void project(const cx<R> p[4], cx<R>& h0, cx<R>& h1) {
    if constexpr (MU == 0) {  // h0 = p0 - SIG i p3, h1 = p1 - SIG i p2
        if constexpr (SIG > 0) {
            h0 = {p[0].re + p[3].im, p[0].im - p[3].re};
            h1 = {p[1].re + p[2].im, p[1].im - p[2].re};
        } else {
            h0 = {p[0].re - p[3].im, p[0].im + p[3].re};
            h1 = {p[1].re - p[2].im, p[1].im + p[2].re};
        }
    } else if constexpr (MU == 1) {  // h0 = p0 - SIG p3, h1 = p1 + SIG p2
        if constexpr (SIG > 0) {
            h0 = csub(p[0], p[3]);
            h1 = cadd(p[1], p[2]);
        } else {
            h0 = cadd(p[0], p[3]);
            h1 = csub(p[1], p[2]);
        }
    } else if constexpr (MU == 2) {  // h0 = p0 - SIG i p2, h1 = p1 + SIG i p3
        if constexpr (SIG > 0) {
            h0 = {p[0].re + p[2].im, p[0].im - p[2].re};
            h1 = {p[1].re - p[3].im, p[1].im + p[3].re};
        } else {
            h0 = {p[0].re - p[2].im, p[0].im + p[2].re};
            h1 = {p[1].re + p[3].im, p[1].im - p[3].re};
        }
    } else {  // h0 = p0 + SIG p2, h1 = p1 + SIG p3
        if constexpr (SIG > 0) {
            h0 = cadd(p[0], p[2]);
            h1 = cadd(p[1], p[3]);
        } else {
            h0 = csub(p[0], p[2]);
            h1 = csub(p[1], p[3]);
        }
    }
}

// acc[0..3] += full spinor rebuilt from the (already transported) half spinor c0, c1.
template <int MU, int SIG, typename R>
__device__ __forceinline__ void reconstruct_add(cx<R> acc[4], cx<R> c0, cx<R> c1) {
    acc[0] = cadd(acc[0], c0);
    acc[1] = cadd(acc[1], c1);
    if constexpr (MU == 0) {  // r2 = SIG i c1, r3 = SIG i c0
        if constexpr (SIG > 0) {
            acc[2] = cadd(acc[2], cmuli(c1));
            acc[3] = cadd(acc[3], cmuli(c0));
        } else {
            acc[2] = csub(acc[2], cmuli(c1));
            acc[3] = csub(acc[3], cmuli(c0));
        }
    } else if constexpr (MU == 1) {  // r2 = SIG c1, r3 = -SIG c0
        if constexpr (SIG > 0) {
            acc[2] = cadd(acc[2], c1);
            acc[3] = csub(acc[3], c0);
        } else {
            acc[2] = csub(acc[2], c1);
            acc[3] = cadd(acc[3], c0);
        }
    } else if constexpr (MU == 2) {  // r2 = SIG i c0, r3 = -SIG i c1
        if constexpr (SIG > 0) {
            acc[2] = cadd(acc[2], cmuli(c0));
            acc[3] = csub(acc[3], cmuli(c1));
        } else {
            acc[2] = csub(acc[2], cmuli(c0));
            acc[3] = cadd(acc[3], cmuli(c1));
        }
    } else {  // r2 = SIG c0, r3 = SIG c1
        if constexpr (SIG > 0) {
            acc[2] = cadd(acc[2], c0);
            acc[3] = cadd(acc[3], c1);
        } else {
            acc[2] = csub(acc[2], c0);
            acc[3] = csub(acc[3], c1);
        }
    }
}

// acc += scale * (1 + SIG g_MU) L u_nb, with L = link (ADJ = false) or link^+ (ADJ = true).
template <int NC, int RB, int MU, int SIG, bool ADJ, class P>
__device__ __forceinline__ void hop(cx<typename P::R> (&acc)[RB][NC][4], const typename P::G* __restrict__ link,
                                    const typename P::S* __restrict__ nb, int nv, typename P::R scale) {
    using R = typename P::R;
    cx<R> l[NC][NC];
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            cx<R> v = io<R, typename P::G>::ld(link + a * NC + b);
            if constexpr (ADJ) {
                l[b][a] = cconj(v);
            } else {
                l[a][b] = v;
            }
        }
#pragma unroll
    for (int k = 0; k < RB; ++k) {
        cx<R> h0[NC], h1[NC];
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            cx<R> p[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) p[s] = io<R, typename P::S>::ld(nb + (b * 4 + s) * nv + k);
            project<MU, SIG>(p, h0[b], h1[b]);
            h0[b] = cscale(scale, h0[b]);
            h1[b] = cscale(scale, h1[b]);
        }
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            cx<R> c0{R(0), R(0)}, c1{R(0), R(0)};
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                cfma(c0, l[a][b], h0[b]);
                cfma(c1, l[a][b], h1[b]);
            }
            reconstruct_add<MU, SIG>(acc[k][a], c0, c1);
        }
    }
}

template <int NC, int RB, int MU, bool DAG, class P>
__device__ __forceinline__ void both_hops(cx<typename P::R> (&acc)[RB][NC][4], const typename P::G* __restrict__ U,
                                          const typename P::S* __restrict__ in, int64_t site, const Coord& c,
                                          const Geom& g, int nv, int r0) {
    using R = typename P::R;
    int64_t fwd, bwd;
    R sf = R(-0.5), sb = R(-0.5);
    if constexpr (MU == 0) {
        fwd = site + (c.x == g.nx - 1 ? 1 - g.nx : 1);
        bwd = site - (c.x == 0 ? 1 - g.nx : 1);
    } else if constexpr (MU == 1) {
        const int64_t st = g.nx;
        fwd = site + (c.y == g.ny - 1 ? (1 - g.ny) * st : st);
        bwd = site - (c.y == 0 ? (1 - g.ny) * st : st);
    } else if constexpr (MU == 2) {
        const int64_t st = static_cast<int64_t>(g.nx) * g.ny;
        fwd = site + (c.z == g.nz - 1 ? (1 - g.nz) * st : st);
        bwd = site - (c.z == 0 ? (1 - g.nz) * st : st);
    } else {
        const int64_t st = static_cast<int64_t>(g.nx) * g.ny * g.nz;
        fwd = site + (c.t == g.nt - 1 ? (1 - g.nt) * st : st);
        bwd = site - (c.t == 0 ? (1 - g.nt) * st : st);
        if (g.apbc) {
            if (c.t == g.nt - 1) sf = R(0.5);
            if (c.t == 0) sb = R(0.5);
        }
    }
    const int64_t vs = static_cast<int64_t>(NC) * 4 * nv;
    constexpr int SF = DAG ? 1 : -1;  // forward projector 1 + SF g_mu
    hop<NC, RB, MU, SF, false, P>(acc, U + (site * 4 + MU) * NC * NC, in + fwd * vs + r0, nv, sf);
    hop<NC, RB, MU, -SF, true, P>(acc, U + (bwd * 4 + MU) * NC * NC, in + bwd * vs + r0, nv, sb);
}

template <int NC, int RB, bool DAG, class P>
__global__ __launch_bounds__(256) void wilson_kernel(const typename P::G* __restrict__ U,
                                                      const typename P::S* __restrict__ in,
                                                      typename P::S* __restrict__ out, typename P::R diag, Geom g,
                                                      int nv) {
    using R = typename P::R;
    const int nrg = nv / RB;
    const int64_t gid = logical_block() * blockDim.x + threadIdx.x;
    if (gid >= g.vol * nrg) return;
    const int64_t site = gid / nrg;
    const int r0 = static_cast<int>(gid - site * nrg) * RB;
    const Coord c = site_coord(site, g);
    const int64_t vs = static_cast<int64_t>(NC) * 4 * nv;

    cx<R> acc[RB][NC][4];
    const typename P::S* centre = in + site * vs + r0;
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[k][a][s] = cscale(diag, io<R, typename P::S>::ld(centre + (a * 4 + s) * nv + k));

    both_hops<NC, RB, 0, DAG, P>(acc, U, in, site, c, g, nv, r0);
    both_hops<NC, RB, 1, DAG, P>(acc, U, in, site, c, g, nv, r0);
    both_hops<NC, RB, 2, DAG, P>(acc, U, in, site, c, g, nv, r0);
    both_hops<NC, RB, 3, DAG, P>(acc, U, in, site, c, g, nv, r0);

    typename P::S* o = out + site * vs + r0;
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int s = 0; s < 4; ++s) io<R, typename P::S>::st(o + (a * 4 + s) * nv + k, acc[k][a][s]);
}

template <int NC, int RB, class P>
void launch_rb(const StencilArgs& a, hipStream_t st) {
    using R = typename P::R;
    const int block = 256;
    const int64_t threads = a.g.vol * (a.nv / RB);
    const dim3 grid(static_cast<unsigned>(grid_blocks_x8(threads, block)));
    const R diag = static_cast<R>(4.0 + a.mass);
    auto U = static_cast<const typename P::G*>(a.gauge);
    auto in = static_cast<const typename P::S*>(a.in);
    auto out = static_cast<typename P::S*>(a.out);
    if (a.dagger)
        hipLaunchKernelGGL((wilson_kernel<NC, RB, true, P>), grid, dim3(block), 0, st, U, in, out, diag, a.g, a.nv);
    else
        hipLaunchKernelGGL((wilson_kernel<NC, RB, false, P>), grid, dim3(block), 0, st, U, in, out, diag, a.g, a.nv);
}

template <int NC, class P>
void launch_nc(const StencilArgs& a, hipStream_t st) {
    switch (a.rb) {
        case 4: launch_rb<NC, 4, P>(a, st); break;
        case 2: launch_rb<NC, 2, P>(a, st); break;
        default: launch_rb<NC, 1, P>(a, st); break;
    }
}

template <class P>
int launch_prec(const StencilArgs& a, hipStream_t st) {
    switch (a.nc) {
        case 1: launch_nc<1, P>(a, st); break;
        case 2: launch_nc<2, P>(a, st); break;
        case 3: launch_nc<3, P>(a, st); break;
        case 4: launch_nc<4, P>(a, st); break;
        default: return DIRAC_EUNSUPPORTED;
    }
    return DIRAC_OK;
}

}  // namespace

int launch_wilson(const StencilArgs& a, hipStream_t st) {
    switch (a.prec) {
        case DIRAC_FP64: return launch_prec<PrecF64>(a, st);
        case DIRAC_FP32: return launch_prec<PrecF32>(a, st);
        case DIRAC_BF16: return launch_prec<PrecBF16>(a, st);
    }
    return DIRAC_EINVAL;
}

}  // namespace dirac
