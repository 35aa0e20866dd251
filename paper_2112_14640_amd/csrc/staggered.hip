// Susskind (staggered) Dirac operator D_S and its adjoint (Sec. 7, Eq. def_stag).
//
//   (D_S u)(n)   = m u(n) + 1/2 sum_mu eta_mu(n) [U_mu(n) u(n+mu) - U_mu(n-mu)^+ u(n-mu)]
//   (D_S^+ u)(n) = m u(n) - 1/2 sum_mu eta_mu(n) [U_mu(n) u(n+mu) - U_mu(n-mu)^+ u(n-mu)]
//
// eta_mu(n) = (-1)^(x_0 + ... + x_{mu-1}) on 0-based coordinates.  One thread owns a site
// and RB consecutive right-hand sides, so each link is loaded once per RB columns.
//
// The same kernels apply the Wilson Laplacian of Eq. app_wlap (flag lap):
//   (-1/2 Delta^std + m^2/2) u(n) = (4 + m^2/2) u(n) - 1/2 sum_mu [U_mu(n) u(n+mu) + U_mu(n-mu)^+ u(n-mu)],
// which acts on colour only: a Wilson-layout vector [colour][spin][rhs] is a colour vector with 4 N_v
// columns.  With lap every hop has the coefficient -1/2 and no phase; the caller passes the diagonal.
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "tile.h"

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
                                                         int nv, SiteOrder order, int lap) {
    using R = typename P::R;
    const int nrg = nv / RB;
    const int64_t gid = logical_block() * blockDim.x + threadIdx.x;
    if (gid >= g.vol * nrg) return;
    const int64_t idx = gid / nrg;
    const int r0 = static_cast<int>(gid - idx * nrg) * RB;
    const int64_t site = ordered_site(idx, order, g);
    const Coord c = site_coord(site, g);
    const int64_t vs = static_cast<int64_t>(NC) * nv;

    cx<R> acc[RB][NC];
    const typename P::S* centre = in + site * vs + r0;
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
        for (int a = 0; a < NC; ++a) acc[k][a] = cscale(mass, io<R, typename P::S>::ld(centre + a * nv + k));

    const R half = lap ? R(-0.5) : (DAG ? R(-0.5) : R(0.5));
    const R bsign = lap ? R(1) : R(-1);  // backward hop coefficient relative to the forward one
    const int par[4] = {0, c.x & 1, (c.x + c.y) & 1, (c.x + c.y + c.z) & 1};
    const int64_t stride[4] = {1, g.nx, static_cast<int64_t>(g.nx) * g.ny, static_cast<int64_t>(g.nx) * g.ny * g.nz};
    const int coord[4] = {c.x, c.y, c.z, c.t};
    const int ext[4] = {g.nx, g.ny, g.nz, g.nt};
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const R eta = (par[mu] && !lap) ? -half : half;
        const int64_t fwd = site + (coord[mu] == ext[mu] - 1 ? (1 - ext[mu]) * stride[mu] : stride[mu]);
        const int64_t bwd = site - (coord[mu] == 0 ? (1 - ext[mu]) * stride[mu] : stride[mu]);
        R sf = eta, sb = bsign * eta;
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


// Row-tiled variant: one x-row (every RHS) per work-group, the rows one step along +-y, +-z,
// +-t staged in LDS one at a time with contiguous loads of Unit (16 or 8 bytes), the next row copy
// and its link in flight while the current direction is consumed (see the Wilson row kernel).
template <int NC, int RB, bool DAG, class P, typename Unit, bool LL>
__global__ __launch_bounds__(512) void staggered_rows_kernel(const typename P::G* __restrict__ U,
                                                             const typename P::S* __restrict__ in,
                                                             typename P::S* __restrict__ out, typename P::R mass,
                                                             Geom g, int nv, RowTile rt, int lap, Epilogue epi) {
    using R = typename P::R;
    using S = typename P::S;
    using G = typename P::G;
    constexpr int PER = NC * RB * static_cast<int>(sizeof(S)) / static_cast<int>(sizeof(Unit));
    constexpr int L = NC * NC;
    extern __shared__ __align__(16) unsigned char sraw[];
    Unit* rtile = reinterpret_cast<Unit*>(sraw);

    const int64_t tix = logical_block();
    if (tix >= rt.ntiles) return;
    const RowPos pos = tile_row_pos(static_cast<uint32_t>(tix), rt, g);
    const uint32_t rho = row_index(pos, g);
    const uint32_t tid = threadIdx.x;
    const bool active = tid < static_cast<uint32_t>(rt.threads);
    const uint32_t tt = active ? tid : tid - rt.threads;
    const uint32_t j = fast_div(tt, rt.magic_nrg);
    const int rg = static_cast<int>(tt - j * rt.nrg);
    const int x = static_cast<int>(j);
    const int64_t rowsite = static_cast<int64_t>(rho) * g.nx;
    const int64_t site = rowsite + x;
    const int cy = pos.y, cz = pos.z, ct = pos.t;
    const Unit* src = reinterpret_cast<const Unit*>(in);
    // sites of the row copy padded to a bank-conflict-free stride
    const uint32_t PADU = row_pad(rt.units, static_cast<uint32_t>(nv) * static_cast<uint32_t>(sizeof(S)) / 4u,
                                  static_cast<uint32_t>(sizeof(Unit)) / 4u);
    const uint32_t SU = rt.units + PADU;  // units per site of the row copy
    uint32_t slot[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const uint32_t u = k * static_cast<uint32_t>(rt.threads) + tt;
        slot[k] = u + fast_div(u, rt.magic_units) * PADU;
    }
    Unit pre[PER];
    const uint32_t row_bytes = static_cast<uint32_t>(rt.row_units * sizeof(Unit));
    auto fetch = [&](int64_t row_start) __attribute__((always_inline)) {
        const auto r = raw_buffer(src + row_start * rt.units, row_bytes);
#pragma unroll
        for (int k = 0; k < PER; ++k)
            pre[k] = buffer_load_unit<Unit>(r, tt * static_cast<uint32_t>(sizeof(Unit)),
                                            static_cast<uint32_t>(k * rt.threads * sizeof(Unit)));
    };
    auto stash = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < PER; ++k) rtile[slot[k]] = pre[k];
    };
    auto at = [&](uint32_t jj) __attribute__((always_inline)) {
        return reinterpret_cast<const S*>(rtile + jj * SU) + rg * RB;
    };
    auto load_link = [&](cx<R> (&l)[NC][NC], const G* lp, bool adj) __attribute__((always_inline)) {
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                const cx<R> v = io<R, G>::ld(lp + a * NC + b);
                if (adj)
                    l[b][a] = cconj(v);
                else
                    l[a][b] = v;
            }
    };
    // LL: the links of the direction being consumed are staged in LDS after the row tile (one
    // N_c x N_c block per site; forward hops the row's own links, backward hops the neighbour
    // row's, used as adjoints), at most LPER complex entries per thread; otherwise every thread
    // loads its own link one direction ahead.
    constexpr int LPER = 2;
    G* lwin = reinterpret_cast<G*>(sraw + (static_cast<size_t>(rt.S) * SU * sizeof(Unit) + 15) / 16 * 16);
    const uint32_t nlink = static_cast<uint32_t>(rt.S) * L;
    G lpre[LPER];
    auto lfetch = [&](int64_t lrow, int mu) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < LPER; ++k) {
            const uint32_t u = k * static_cast<uint32_t>(rt.threads) + tt;
            if (u < nlink) {
                const uint32_t sx = u / L;
                lpre[k] = U[((lrow + sx) * 4 + mu) * L + (u - sx * L)];
            }
        }
    };
    auto lstash = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < LPER; ++k) {
            const uint32_t u = k * static_cast<uint32_t>(rt.threads) + tt;
            if (u < nlink) lwin[u] = lpre[k];
        }
    };
    cx<R> acc[RB][NC];
    const R half = lap ? R(-0.5) : (DAG ? R(-0.5) : R(0.5));
    const R bsign = lap ? R(1) : R(-1);  // backward hop coefficient relative to the forward one
    // eta_mu(n) = (-1)^(x_0 + ... + x_{mu-1}) (all 1 for the Laplacian)
    const R eta[4] = {half, ((x & 1) && !lap) ? -half : half, (((x + cy) & 1) && !lap) ? -half : half,
                      (((x + cy + cz) & 1) && !lap) ? -half : half};
    const int xp = x + 1 == g.nx ? 0 : x + 1;
    const int xm = x == 0 ? g.nx - 1 : x - 1;
    cx<R> lxp[NC][NC], lxm[NC][NC], lnext[NC][NC];
    fetch(rowsite);
    if constexpr (LL) {
        lfetch(rowsite, 0);
    } else {
        load_link(lxp, U + (site * 4 + 0) * L, false);
        load_link(lxm, U + ((rowsite + xm) * 4 + 0) * L, true);
    }
    stash();
    if constexpr (LL) lstash();
    __syncthreads();
    fetch(row_neighbour_start(pos, 0, g));
    if constexpr (LL) {
        lfetch(rowsite, 1);
        load_link(lxp, lwin + x * L, false);
        load_link(lxm, lwin + xm * L, true);
    } else {
        load_link(lnext, U + (site * 4 + 1) * L, false);
    }
    auto hop_acc = [&](const cx<R> (&l)[NC][NC], const S* nb, R scale) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            cx<R> p[NC];
#pragma unroll
            for (int b = 0; b < NC; ++b) p[b] = cscale(scale, io<R, S>::ld(nb + b * nv + k));
#pragma unroll
            for (int a = 0; a < NC; ++a)
#pragma unroll
                for (int b = 0; b < NC; ++b) cfma(acc[k][a], l[a][b], p[b]);
        }
    };
    if (active) {
        const S* mine = at(j);
#pragma unroll
        for (int k = 0; k < RB; ++k)
#pragma unroll
            for (int a = 0; a < NC; ++a) acc[k][a] = cscale(mass, io<R, S>::ld(mine + a * nv + k));
        hop_acc(lxp, at(xp), eta[0]);
        hop_acc(lxm, at(xm), bsign * eta[0]);
    }
    auto step = [&](auto mu_c, auto back_c) __attribute__((always_inline)) {
        constexpr int MU = decltype(mu_c)::value;
        constexpr bool BACK = decltype(back_c)::value;
        constexpr int DIR = 2 * (MU - 1) + (BACK ? 1 : 0);
        cx<R> lcur[NC][NC];
        if constexpr (!LL) {
#pragma unroll
            for (int a = 0; a < NC; ++a)
#pragma unroll
                for (int b = 0; b < NC; ++b) lcur[a][b] = lnext[a][b];
        }
        __syncthreads();
        stash();
        if constexpr (LL) lstash();
        __syncthreads();
        if constexpr (DIR < 5) {
            constexpr int ND = DIR + 1;
            constexpr int NMU = ND / 2 + 1;
            const int64_t nrow = row_neighbour_start(pos, ND, g);
            fetch(nrow);
            if constexpr (LL)
                lfetch(ND % 2 == 0 ? rowsite : nrow, NMU);
            else if constexpr (ND % 2 == 0)
                load_link(lnext, U + (site * 4 + NMU) * L, false);
            else
                load_link(lnext, U + ((nrow + x) * 4 + NMU) * L, true);
        }
        if constexpr (LL) load_link(lcur, lwin + x * L, BACK);
        if (active) {
            R sc = BACK ? bsign * eta[MU] : eta[MU];
            if (MU == 3 && g.apbc && ct == (BACK ? 0 : g.nt - 1)) sc = -sc;  // fermion sign
            hop_acc(lcur, at(j), sc);
        }
    };
    step(std::integral_constant<int, 1>{}, std::false_type{});
    step(std::integral_constant<int, 1>{}, std::true_type{});
    step(std::integral_constant<int, 2>{}, std::false_type{});
    step(std::integral_constant<int, 2>{}, std::true_type{});
    step(std::integral_constant<int, 3>{}, std::false_type{});
    step(std::integral_constant<int, 3>{}, std::true_type{});
    if (epi.mode == 2) {  // r -= alpha (D^+ t): the output itself is not written
        row_epilogue<RB, NC, R, S>(epi, acc, active, site * (NC * nv) + rg * RB, nv, rg * RB, j, rt.S, tix,
                                   reinterpret_cast<double*>(sraw));
        return;
    }
    __syncthreads();
    if (active) {
        S* o = const_cast<S*>(at(j));
#pragma unroll
        for (int k = 0; k < RB; ++k)
#pragma unroll
            for (int a = 0; a < NC; ++a) io<R, S>::st(o + a * nv + k, acc[k][a]);
    }
    __syncthreads();
    Unit* dst = reinterpret_cast<Unit*>(out) + rowsite * rt.units;
    const uint32_t total = static_cast<uint32_t>(rt.S) * rt.units;
    // streaming stores: the output is not read again by this launch, so its lines should not
    // displace input rows that neighbouring work-groups still read from L2
    for (uint32_t u = tid; u < total; u += blockDim.x)
        __builtin_nontemporal_store(rtile[u + fast_div(u, rt.magic_units) * PADU], dst + u);
    if (epi.mode == 1)
        row_epilogue<RB, NC, R, S>(epi, acc, active, 0, nv, rg * RB, j, rt.S, tix, reinterpret_cast<double*>(sraw));
}

template <int NC, int RB, class P>
bool launch_rows(const StencilArgs& a, int nv, typename P::R diag, hipStream_t st) {
    using S = typename P::S;
    constexpr size_t share = static_cast<size_t>(NC) * RB * sizeof(S);  // bytes per thread per row copy
    constexpr size_t ub = share % 16 == 0 ? 16 : (share % 8 == 0 ? 8 : 0);
    if constexpr (ub == 0) {
        return false;
    } else {
        using Unit = std::conditional_t<ub == 16, u32x4, u32x2>;
        const size_t block_bytes = static_cast<size_t>(NC) * nv * sizeof(S);
        if (block_bytes % ub != 0 || !tile_aligned(a)) return false;
        const int units = static_cast<int>(block_bytes / ub);
        const int nrg = nv / RB;
        const int64_t rows = a.g.vol / a.g.nx;
        const int64_t threads = static_cast<int64_t>(a.g.nx) * nrg;
        const uint32_t pad = row_pad(units, static_cast<uint32_t>(nv * sizeof(S) / 4), static_cast<uint32_t>(ub / 4));
        const size_t lds = static_cast<size_t>(a.g.nx) * (units + pad) * ub;
        if (threads < 64 || threads > 512 || lds > 64 * 1024) return false;
        RowTile rt{};
        rt.R = 1;
        rt.S = a.g.nx;
        rt.nrg = nrg;
        rt.units = units;
        rt.row_units = a.g.nx * units;
        rt.threads = static_cast<int>(threads);
        rt.ntiles = rows;
        rt.nseg = 1;
        rt.magic_nrg = div_magic(nrg);
        rt.magic_nx = div_magic(a.g.nx);
        rt.magic_units = div_magic(units);
        rt.magic_row_units = div_magic(rt.row_units);
        if (!row_order(4, a.g, rt)) return false;
        const int block = (rt.threads + 63) / 64 * 64;
        const dim3 grid(static_cast<unsigned>(grid_blocks_x8(rt.ntiles, 1)));
        auto U = static_cast<const typename P::G*>(a.gauge);
        auto in = static_cast<const S*>(a.in);
        auto out = static_cast<S*>(a.out);
        const int lap = a.laplace ? 1 : 0;
        // FP32 and BF16: each direction's links staged in LDS after the row tile (at most two entries
        // per thread); FP64 loads them per thread (its staged form touched scratch and ran slower)
        const size_t lds_ll = (lds + 15) / 16 * 16 + static_cast<size_t>(a.g.nx) * NC * NC * sizeof(typename P::G);
        const bool ll = sizeof(typename P::R) == 4 && static_cast<int64_t>(a.g.nx) * NC * NC <= 2 * threads &&
                        lds_ll <= 64 * 1024;
        if (ll) {
            if (a.dagger)
                hipLaunchKernelGGL((staggered_rows_kernel<NC, RB, true, P, Unit, true>), grid, dim3(block), lds_ll, st,
                                   U, in, out, diag, a.g, nv, rt, lap, a.epi);
            else
                hipLaunchKernelGGL((staggered_rows_kernel<NC, RB, false, P, Unit, true>), grid, dim3(block), lds_ll, st,
                                   U, in, out, diag, a.g, nv, rt, lap, a.epi);
        } else if (a.dagger) {
            hipLaunchKernelGGL((staggered_rows_kernel<NC, RB, true, P, Unit, false>), grid, dim3(block), lds, st, U, in,
                               out, diag, a.g, nv, rt, lap, a.epi);
        } else {
            hipLaunchKernelGGL((staggered_rows_kernel<NC, RB, false, P, Unit, false>), grid, dim3(block), lds, st, U,
                               in, out, diag, a.g, nv, rt, lap, a.epi);
        }
        return true;
    }
}

// false: an epilogue was asked for and only the direct kernel could take this shape (nothing launched)
template <int NC, int RB, class P>
bool launch_rb(const StencilArgs& a, hipStream_t st) {
    using R = typename P::R;
    // the Wilson Laplacian treats the spin index as four more columns per colour
    const int nv = a.laplace ? 4 * a.nv : a.nv;
    const R diag = static_cast<R>(a.laplace ? 4.0 + 0.5 * a.mass * a.mass : a.mass);
    if (a.variant == 4 && launch_rows<NC, RB, P>(a, nv, diag, st)) return true;
    if (a.epi.mode != 0) return false;
    const int block = 256;
    const int64_t threads = a.g.vol * (nv / RB);
    const dim3 grid(static_cast<unsigned>(grid_blocks_x8(threads, block)));
    auto U = static_cast<const typename P::G*>(a.gauge);
    auto in = static_cast<const typename P::S*>(a.in);
    auto out = static_cast<typename P::S*>(a.out);
    const SiteOrder ord = make_site_order(a.g);
    const int lap = a.laplace ? 1 : 0;
    if (a.dagger)
        hipLaunchKernelGGL((staggered_kernel<NC, RB, true, P>), grid, dim3(block), 0, st, U, in, out, diag, a.g, nv,
                           ord, lap);
    else
        hipLaunchKernelGGL((staggered_kernel<NC, RB, false, P>), grid, dim3(block), 0, st, U, in, out, diag, a.g, nv,
                           ord, lap);
    return true;
}

template <int NC, class P>
bool launch_nc(const StencilArgs& a, hipStream_t st) {
    switch (a.rb) {
        case 4: return launch_rb<NC, 4, P>(a, st);
        case 2: return launch_rb<NC, 2, P>(a, st);
        default: return launch_rb<NC, 1, P>(a, st);
    }
}

template <class P>
int launch_prec(const StencilArgs& a, hipStream_t st) {
    bool ok;
    switch (a.nc) {
        case 1: ok = launch_nc<1, P>(a, st); break;
        case 2: ok = launch_nc<2, P>(a, st); break;
        case 3: ok = launch_nc<3, P>(a, st); break;
        case 4: ok = launch_nc<4, P>(a, st); break;
        default: return DIRAC_EUNSUPPORTED;
    }
    return ok ? DIRAC_OK : kNoEpilogue;
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
