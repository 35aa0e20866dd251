// Susskind (staggered) Dirac operator D_S and its adjoint (Sec. 7, Eq. def_stag).
//
//   (D_S u)(n)   = m u(n) + 1/2 sum_mu eta_mu(n) [U_mu(n) u(n+mu) - U_mu(n-mu)^+ u(n-mu)]
//   (D_S^+ u)(n) = m u(n) - 1/2 sum_mu eta_mu(n) [U_mu(n) u(n+mu) - U_mu(n-mu)^+ u(n-mu)]
//
// eta_mu(n) = (-1)^(x_0 + ... + x_{mu-1}) on 0-based coordinates.  One thread owns a site
// and RB consecutive right-hand sides, so each link is loaded once per RB columns.
#include "common.h"
#include "kernels.h"

namespace dirac {

namespace {

template <int NC, int RB, bool ADJ, class P>
__device__ __forceinline__ void stag_hop(cx<typename P::R> (&acc)[RB][NC], const typename P::G* __restrict__ link,
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
        cx<R> p[NC];
#pragma unroll
        for (int b = 0; b < NC; ++b) p[b] = cscale(scale, io<R, typename P::S>::ld(nb + b * nv + k));
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int b = 0; b < NC; ++b) cfma(acc[k][a], l[a][b], p[b]);
    }
}

template <int NC, int RB, bool DAG, class P>
__global__ __launch_bounds__(256) void staggered_kernel(const typename P::G* __restrict__ U,
                                                         const typename P::S* __restrict__ in,
                                                         typename P::S* __restrict__ out, typename P::R mass, Geom g,
                                                         int nv) {
    using R = typename P::R;
    const int nrg = nv / RB;
    const int64_t gid = logical_block() * blockDim.x + threadIdx.x;
    if (gid >= g.vol * nrg) return;
    const int64_t site = gid / nrg;
    const int r0 = static_cast<int>(gid - site * nrg) * RB;
    const Coord c = site_coord(site, g);
    const int64_t vs = static_cast<int64_t>(NC) * nv;

    cx<R> acc[RB][NC];
    const typename P::S* centre = in + site * vs + r0;
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
        for (int a = 0; a < NC; ++a) acc[k][a] = cscale(mass, io<R, typename P::S>::ld(centre + a * nv + k));

    const R half = DAG ? R(-0.5) : R(0.5);
    const int par[4] = {0, c.x & 1, (c.x + c.y) & 1, (c.x + c.y + c.z) & 1};
    const int64_t stride[4] = {1, g.nx, static_cast<int64_t>(g.nx) * g.ny, static_cast<int64_t>(g.nx) * g.ny * g.nz};
    const int coord[4] = {c.x, c.y, c.z, c.t};
    const int ext[4] = {g.nx, g.ny, g.nz, g.nt};
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const R eta = par[mu] ? -half : half;
        const int64_t fwd = site + (coord[mu] == ext[mu] - 1 ? (1 - ext[mu]) * stride[mu] : stride[mu]);
        const int64_t bwd = site - (coord[mu] == 0 ? (1 - ext[mu]) * stride[mu] : stride[mu]);
        R sf = eta, sb = -eta;
        if (mu == 3 && g.apbc) {
            if (c.t == g.nt - 1) sf = -sf;
            if (c.t == 0) sb = -sb;
        }
        stag_hop<NC, RB, false, P>(acc, U + (site * 4 + mu) * NC * NC, in + fwd * vs + r0, nv, sf);
        stag_hop<NC, RB, true, P>(acc, U + (bwd * 4 + mu) * NC * NC, in + bwd * vs + r0, nv, sb);
    }

    typename P::S* o = out + site * vs + r0;
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
        for (int a = 0; a < NC; ++a) io<R, typename P::S>::st(o + a * nv + k, acc[k][a]);
}

template <int NC, int RB, class P>
void launch_rb(const StencilArgs& a, hipStream_t st) {
    using R = typename P::R;
    const int block = 256;
    const int64_t threads = a.g.vol * (a.nv / RB);
    const dim3 grid(static_cast<unsigned>(grid_blocks_x8(threads, block)));
    auto U = static_cast<const typename P::G*>(a.gauge);
    auto in = static_cast<const typename P::S*>(a.in);
    auto out = static_cast<typename P::S*>(a.out);
    const R m = static_cast<R>(a.mass);
    if (a.dagger)
        hipLaunchKernelGGL((staggered_kernel<NC, RB, true, P>), grid, dim3(block), 0, st, U, in, out, m, a.g, a.nv);
    else
        hipLaunchKernelGGL((staggered_kernel<NC, RB, false, P>), grid, dim3(block), 0, st, U, in, out, m, a.g, a.nv);
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

int launch_staggered(const StencilArgs& a, hipStream_t st) {
    switch (a.prec) {
        case DIRAC_FP64: return launch_prec<PrecF64>(a, st);
        case DIRAC_FP32: return launch_prec<PrecF32>(a, st);
        case DIRAC_BF16: return launch_prec<PrecBF16>(a, st);
    }
    return DIRAC_EINVAL;
}

}  // namespace dirac
