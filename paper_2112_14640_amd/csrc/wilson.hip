// Wilson Dirac operator D_W and its adjoint (Sec. 5, Eq. app_wils; r = 1), with the optional clover
// term C of Eq. def_clov added at the site (C is hermitian, so (D_W + C)^+ = D_W^+ + C):
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
#include <type_traits>

#include "clover.h"
#include "common.h"
#include "kernels.h"
#include "tile.h"

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

// acc[0..3] += s * (full spinor rebuilt from c0, c1): the scale rides on the multiply-adds.
template <int MU, int SIG, typename R>
__device__ __forceinline__ void reconstruct_scaled(cx<R> acc[4], cx<R> c0, cx<R> c1, R s) {
    // a += f v and a += f i v (i v = (-v.im, v.re)), f = +-s
    auto ax = [](cx<R>& a, R f, cx<R> v) __attribute__((always_inline)) {
        a.re += f * v.re;
        a.im += f * v.im;
    };
    auto axi = [](cx<R>& a, R f, cx<R> v) __attribute__((always_inline)) {
        a.re -= f * v.im;
        a.im += f * v.re;
    };
    const R n = -s;
    ax(acc[0], s, c0);
    ax(acc[1], s, c1);
    if constexpr (MU == 0) {  // r2 = SIG i c1, r3 = SIG i c0
        axi(acc[2], SIG > 0 ? s : n, c1);
        axi(acc[3], SIG > 0 ? s : n, c0);
    } else if constexpr (MU == 1) {  // r2 = SIG c1, r3 = -SIG c0
        ax(acc[2], SIG > 0 ? s : n, c1);
        ax(acc[3], SIG > 0 ? n : s, c0);
    } else if constexpr (MU == 2) {  // r2 = SIG i c0, r3 = -SIG i c1
        axi(acc[2], SIG > 0 ? s : n, c0);
        axi(acc[3], SIG > 0 ? n : s, c1);
    } else {  // r2 = SIG c0, r3 = SIG c1
        ax(acc[2], SIG > 0 ? s : n, c0);
        ax(acc[3], SIG > 0 ? s : n, c1);
    }
}

// L = link (ADJ = false) or link^+ (ADJ = true) into registers.
template <int NC, bool ADJ, class P>
__device__ __forceinline__ void load_link(cx<typename P::R> (&l)[NC][NC], const typename P::G* __restrict__ link) {
    using R = typename P::R;
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
}

// acc += scale * (1 + SIG g_MU) L u_nb for a link matrix L already in registers.  NVC > 0 fixes
// the RHS stride at compile time (else nv).
template <int NC, int RB, int MU, int SIG, class P, int NVC = 0>
__device__ __forceinline__ void hop_with(cx<typename P::R> (&acc)[RB][NC][4], const cx<typename P::R> (&l)[NC][NC],
                                         const typename P::S* __restrict__ nb, int nv, typename P::R scale) {
    using R = typename P::R;
    const int stride = NVC > 0 ? NVC : nv;
#pragma unroll
    for (int k = 0; k < RB; ++k) {
        cx<R> h0[NC], h1[NC];
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            cx<R> p[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) p[s] = io<R, typename P::S>::ld(nb + (b * 4 + s) * stride + k);
            project<MU, SIG>(p, h0[b], h1[b]);
        }
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            cx<R> c0{R(0), R(0)}, c1{R(0), R(0)};
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                cfma(c0, l[a][b], h0[b]);
                cfma(c1, l[a][b], h1[b]);
            }
            reconstruct_scaled<MU, SIG>(acc[k][a], c0, c1, scale);
        }
    }
}

// Direction-generic hop (runtime mu and projector sign, wave-uniform).  With P = 1 + sig g_mu
// in the chiral basis the half spinor is h0 = p0 + c0 p_A, h1 = p1 + c1 p_B and the full spinor
// is rebuilt as (h0, h1, e2 h_C, e3 h_D), where every c, e is one of +-1, +-i:
//   mu=0: A,B = 3,2  c0,c1 = -sig i, -sig i   C,D = 1,0  e2,e3 = sig i, sig i
//   mu=1: A,B = 3,2  c0,c1 = -sig, +sig       C,D = 1,0  e2,e3 = sig, -sig
//   mu=2: A,B = 2,3  c0,c1 = -sig i, +sig i   C,D = 0,1  e2,e3 = sig i, -sig i
//   mu=3: A,B = 2,3  c0,c1 = +sig, +sig       C,D = 0,1  e2,e3 = sig, sig
struct UnitC {
    int re, im;
};
template <typename R>
__device__ __forceinline__ cx<R> umul(UnitC u, cx<R> x) {
    // (u.re + i u.im)(x.re + i x.im), u one of +-1, +-i
    return {R(u.re) * x.re - R(u.im) * x.im, R(u.re) * x.im + R(u.im) * x.re};
}

template <int NC, int RB, class P>
__device__ __forceinline__ void hop_rt(cx<typename P::R> (&acc)[RB][NC][4], const typename P::G* __restrict__ link,
                                       bool adj, const typename P::S* __restrict__ nb, int nv, typename P::R scale,
                                       int mu, int sig) {
    using R = typename P::R;
    const bool lo = mu < 2;
    UnitC c0, c1, e2, e3;
    switch (mu) {
        case 0: c0 = {0, -sig}; c1 = {0, -sig}; e2 = {0, sig}; e3 = {0, sig}; break;
        case 1: c0 = {-sig, 0}; c1 = {sig, 0}; e2 = {sig, 0}; e3 = {-sig, 0}; break;
        case 2: c0 = {0, -sig}; c1 = {0, sig}; e2 = {0, sig}; e3 = {0, -sig}; break;
        default: c0 = {sig, 0}; c1 = {sig, 0}; e2 = {sig, 0}; e3 = {sig, 0}; break;
    }
    cx<R> l[NC][NC];
    if (adj) {
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int b = 0; b < NC; ++b) l[b][a] = cconj(io<R, typename P::G>::ld(link + a * NC + b));
    } else {
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int b = 0; b < NC; ++b) l[a][b] = io<R, typename P::G>::ld(link + a * NC + b);
    }
#pragma unroll
    for (int k = 0; k < RB; ++k) {
        cx<R> h0[NC], h1[NC];
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            cx<R> p[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) p[s] = io<R, typename P::S>::ld(nb + (b * 4 + s) * nv + k);
            const cx<R> pa = lo ? p[3] : p[2];
            const cx<R> pb = lo ? p[2] : p[3];
            h0[b] = cscale(scale, cadd(p[0], umul(c0, pa)));
            h1[b] = cscale(scale, cadd(p[1], umul(c1, pb)));
        }
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            cx<R> x0{R(0), R(0)}, x1{R(0), R(0)};
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                cfma(x0, l[a][b], h0[b]);
                cfma(x1, l[a][b], h1[b]);
            }
            acc[k][a][0] = cadd(acc[k][a][0], x0);
            acc[k][a][1] = cadd(acc[k][a][1], x1);
            acc[k][a][2] = cadd(acc[k][a][2], umul(e2, lo ? x1 : x0));
            acc[k][a][3] = cadd(acc[k][a][3], umul(e3, lo ? x0 : x1));
        }
    }
}

// Direct form: one thread per (site, RB right-hand sides), neighbours read from global memory, one
// hop direction per loop iteration (only its loads are live, which keeps the register count and so
// the waves per SIMD moderate).  It serves the shapes the row tiles cannot take.
template <int NC, int RB, bool DAG, class P>
__global__ __launch_bounds__(256) void wilson_kernel(const typename P::G* __restrict__ U,
                                                      const typename P::S* __restrict__ in,
                                                      typename P::S* __restrict__ out, typename P::R diag, Geom g,
                                                      int nv, SiteOrder order, const typename P::R* __restrict__ clov) {
    using R = typename P::R;
    const int nrg = nv / RB;
    const int64_t gid = logical_block() * blockDim.x + threadIdx.x;
    if (gid >= g.vol * nrg) return;
    const int64_t idx = gid / nrg;
    const int r0 = static_cast<int>(gid - idx * nrg) * RB;
    const int64_t site = ordered_site(idx, order, g);
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
    if (clov) clover_add<NC, RB>(acc, centre, nv, clov + site * clover_reals<NC>());

    const int co[4] = {c.x, c.y, c.z, c.t};
    const int ext[4] = {g.nx, g.ny, g.nz, g.nt};
#pragma nounroll
    for (int d = 0; d < 8; ++d) {
        const int mu = d >> 1;
        const bool back = d & 1;
        const int64_t stride = mu == 0 ? 1 : (mu == 1 ? g.nx : (mu == 2 ? static_cast<int64_t>(g.nx) * g.ny
                                                                         : static_cast<int64_t>(g.nx) * g.ny * g.nz));
        const int cm = mu == 0 ? co[0] : (mu == 1 ? co[1] : (mu == 2 ? co[2] : co[3]));
        const int em = mu == 0 ? ext[0] : (mu == 1 ? ext[1] : (mu == 2 ? ext[2] : ext[3]));
        int64_t nbs;
        R scale = R(-0.5);
        if (!back) {
            nbs = site + (cm == em - 1 ? (1 - em) * stride : stride);
            if (mu == 3 && g.apbc && cm == em - 1) scale = R(0.5);
        } else {
            nbs = site - (cm == 0 ? (1 - em) * stride : stride);
            if (mu == 3 && g.apbc && cm == 0) scale = R(0.5);
        }
        // D: forward (1 - g_mu), backward (1 + g_mu); the adjoint swaps them
        const int sig = (back != DAG) ? 1 : -1;
        const typename P::G* link = U + ((back ? nbs : site) * 4 + mu) * NC * NC;
        hop_rt<NC, RB, P>(acc, link, back, in + nbs * vs + r0, nv, scale, mu, sig);
    }

    typename P::S* o = out + site * vs + r0;
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int s = 0; s < 4; ++s) io<R, typename P::S>::st(o + (a * 4 + s) * nv + k, acc[k][a][s]);
}

// Row-tiled variant (see RowTile).  Seven row copies per tile: the own rows (mass term and the
// +-x hops) and the rows one step away in +y, -y, +z, -z, +t, -t.  The copy of the next
// direction is issued into registers before the current direction is consumed from LDS, so the
// loads of one direction overlap the arithmetic of the previous one.  The output tile leaves
// through LDS as one contiguous store.

template <int NC, int RB, bool DAG, class P, int NVC, bool LL, bool CLOV>
__global__ __launch_bounds__(512) void wilson_rows_kernel(const typename P::G* __restrict__ U,
                                                          const typename P::S* __restrict__ in,
                                                          typename P::S* __restrict__ out, typename P::R diag,
                                                          Geom g, int nv, RowTile rt,
                                                          const typename P::R* __restrict__ clov, Epilogue epi) {
    using R = typename P::R;
    using S = typename P::S;
    constexpr int PER = RowUnits<NC, RB, P>::PER;
    constexpr int L = NC * NC;
    extern __shared__ __align__(16) u32x4 rtile[];

    const int64_t tix = logical_block();
    if (tix >= rt.ntiles) return;
    const RowPos pos = tile_row_pos(static_cast<uint32_t>(tix), rt, g);  // one row per work-group
    const uint32_t rho = row_index(pos, g);
    const uint32_t tid = threadIdx.x;
    const bool active = tid < static_cast<uint32_t>(rt.threads);
    // padding threads (block rounded up to whole wavefronts) shadow a real thread: same loads and
    // LDS writes of the same values, no global store
    const uint32_t tt = active ? tid : tid - rt.threads;
    const uint32_t j = fast_div(tt, rt.magic_nrg);  // x of this thread's site
    const int rg = static_cast<int>(tt - j * rt.nrg);
    const int x = static_cast<int>(j);
    const int64_t rowsite = static_cast<int64_t>(rho) * g.nx;
    const int64_t site = rowsite + x;
    const int ct = pos.t;
    const u32x4* src = reinterpret_cast<const u32x4*>(in);
    if constexpr (NVC > 0) nv = NVC;

    // unit k of this thread: k * threads + tt of the row copy; its padded LDS slot (sites padded to a
    // bank-conflict-free stride)
    const uint32_t PADU = row_pad(rt.units, static_cast<uint32_t>(nv) * static_cast<uint32_t>(sizeof(S)) / 4u);
    const uint32_t SU = rt.units + PADU;  // units per site of the row copy
    uint32_t slot[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const uint32_t u = k * static_cast<uint32_t>(rt.threads) + tt;
        slot[k] = u + fast_div(u, rt.magic_units) * PADU;
    }
    u32x4 pre[PER];
    const uint32_t row_bytes = static_cast<uint32_t>(rt.row_units) * 16u;
    auto fetch = [&](int64_t row_start) __attribute__((always_inline)) {
        const auto r = raw_buffer(src + row_start * rt.units, row_bytes);
#pragma unroll
        for (int k = 0; k < PER; ++k)
            pre[k] = buffer_load_unit<u32x4>(r, tt * 16u, static_cast<uint32_t>(k * rt.threads) * 16u);
    };
    auto stash = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < PER; ++k) rtile[slot[k]] = pre[k];
    };
    auto at = [&](uint32_t jj) __attribute__((always_inline)) {
        return reinterpret_cast<const S*>(rtile + jj * SU) + rg * RB;
    };

    // LL: the links of the direction being consumed are staged in LDS after the row tile, one
    // N_c x N_c block per site of the row (forward hops: the row's own links; backward hops: the
    // neighbour row's, used as adjoints), copied alongside the row; each thread moves at most LPER
    // complex entries (NVC > 0).  Otherwise every thread loads its own link one direction ahead.
    using G = typename P::G;
    constexpr int NRG = NVC > 0 ? NVC / RB : 1;
    constexpr int LPER = LL ? (L + NRG - 1) / NRG : 1;
    G* lwin = reinterpret_cast<G*>(rtile + rt.S * SU);
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

    cx<R> acc[RB][NC][4];
    constexpr int SF = DAG ? 1 : -1;  // forward projector 1 + SF g_mu
    // Links are loaded one direction ahead and before the next row copy: loads complete in issue
    // order, so waiting for a link never waits for the row copy still in flight.
    const int xp = x + 1 == g.nx ? 0 : x + 1;
    const int xm = x == 0 ? g.nx - 1 : x - 1;
    cx<R> lxp[NC][NC], lxm[NC][NC], lnext[NC][NC];
    fetch(rowsite);
    if constexpr (LL) {
        lfetch(rowsite, 0);
    } else {
        load_link<NC, false, P>(lxp, U + (site * 4 + 0) * L);
        load_link<NC, true, P>(lxm, U + ((rowsite + xm) * 4 + 0) * L);
    }
    stash();
    if constexpr (LL) lstash();
    __syncthreads();
    fetch(row_neighbour_start(pos, 0, g));
    auto mass_term = [&]() __attribute__((always_inline)) {
        const S* mine = at(j);
#pragma unroll
        for (int k = 0; k < RB; ++k)
#pragma unroll
            for (int a = 0; a < NC; ++a)
#pragma unroll
                for (int s = 0; s < 4; ++s) acc[k][a][s] = cscale(diag, io<R, S>::ld(mine + (a * 4 + s) * nv + k));
        if constexpr (CLOV) clover_add<NC, RB>(acc, mine, nv, clov + site * clover_reals<NC>());
    };
    // with a clover field the site's clover block is applied from the own row before the x links are
    // taken into registers
    if constexpr (CLOV)
        if (active) mass_term();
    if constexpr (LL) {
        lfetch(rowsite, 1);
        load_link<NC, false, P>(lxp, lwin + x * L);
        load_link<NC, true, P>(lxm, lwin + xm * L);
    } else {
        load_link<NC, false, P>(lnext, U + (site * 4 + 1) * L);
    }
    // each transported half spinor enters the sum with -1/2 (+1/2 across the antiperiodic t
    // boundary) as the multiplier of the rebuild's multiply-adds
    if (active) {
        if constexpr (!CLOV) mass_term();
        hop_with<NC, RB, 0, SF, P, NVC>(acc, lxp, at(xp), nv, R(-0.5));
        hop_with<NC, RB, 0, -SF, P, NVC>(acc, lxm, at(xm), nv, R(-0.5));
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
            if constexpr (LL) {
                lfetch(ND % 2 == 0 ? rowsite : nrow, NMU);
            } else if constexpr (ND % 2 == 0) {
                load_link<NC, false, P>(lnext, U + (site * 4 + NMU) * L);
            } else {
                load_link<NC, true, P>(lnext, U + ((nrow + x) * 4 + NMU) * L);
            }
        }
        if constexpr (LL) load_link<NC, BACK, P>(lcur, lwin + x * L);
        if (active) {
            const bool wrap = MU == 3 && g.apbc && ct == (BACK ? 0 : g.nt - 1);  // fermion sign
            hop_with<NC, RB, MU, (BACK ? -SF : SF), P, NVC>(acc, lcur, at(j), nv,
                                                                        wrap ? R(0.5) : R(-0.5));
        }
    };
    step(std::integral_constant<int, 1>{}, std::false_type{});
    step(std::integral_constant<int, 1>{}, std::true_type{});
    step(std::integral_constant<int, 2>{}, std::false_type{});
    step(std::integral_constant<int, 2>{}, std::true_type{});
    step(std::integral_constant<int, 3>{}, std::false_type{});
    step(std::integral_constant<int, 3>{}, std::true_type{});
    // the thread's outputs as [RB][NC * 4] (element a * 4 + s at offset (a * 4 + s) * nv)
    const auto& flat = reinterpret_cast<const cx<R>(&)[RB][NC * 4]>(acc);
    if (epi.mode == 2) {  // r -= alpha (D^+ t): the output itself is not written
        row_epilogue<RB, NC * 4, R, S>(epi, flat, active, site * (NC * 4 * nv) + rg * RB, nv, rg * RB, j, rt.S, tix,
                                       reinterpret_cast<double*>(rtile));
        return;
    }
    __syncthreads();
    if (active) {
        S* o = const_cast<S*>(at(j));
#pragma unroll
        for (int k = 0; k < RB; ++k)
#pragma unroll
            for (int a = 0; a < NC; ++a)
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    io<R, S>::st(o + (a * 4 + s) * nv + k, acc[k][a][s]);
    }
    __syncthreads();
    u32x4* dst = reinterpret_cast<u32x4*>(out) + rowsite * rt.units;
    const uint32_t total = static_cast<uint32_t>(rt.S) * rt.units;
    // streaming stores: the output is not read again by this launch, so its lines should not
    // displace input rows that neighbouring work-groups still read from L2
    for (uint32_t u = tid; u < total; u += blockDim.x)
        __builtin_nontemporal_store(rtile[u + fast_div(u, rt.magic_units) * PADU], dst + u);
    if (epi.mode == 1)
        row_epilogue<RB, NC * 4, R, S>(epi, flat, active, 0, nv, rg * RB, j, rt.S, tix,
                                       reinterpret_cast<double*>(rtile));
}

template <int NC, int RB, class P>
bool launch_rows(const StencilArgs& a, hipStream_t st) {
    using S = typename P::S;
    const size_t block_bytes = static_cast<size_t>(NC) * 4 * a.nv * sizeof(S);
    if (block_bytes % 16 != 0 || !tile_aligned(a)) return false;
    const int units = static_cast<int>(block_bytes / 16);
    const int nrg = a.nv / RB;
    const int64_t rows = a.g.vol / a.g.nx;
    const uint32_t pad = row_pad(units, static_cast<uint32_t>(a.nv * sizeof(S) / 4));
    const int Rr = choose_tile_rows(a.variant, rows, a.g.nx, units, nrg, pad);
    if (Rr == 0) return false;
    RowTile rt;
    rt.R = Rr;
    rt.S = Rr * a.g.nx;
    rt.nrg = nrg;
    rt.units = units;
    rt.row_units = a.g.nx * units;
    rt.threads = rt.S * nrg;
    rt.ntiles = rows / Rr;
    rt.nseg = 1;
    rt.magic_nrg = div_magic(nrg);
    rt.magic_nx = div_magic(a.g.nx);
    rt.magic_units = div_magic(units);
    rt.magic_row_units = div_magic(rt.row_units);
    if (!row_order(4, a.g, rt)) return false;
    const int block = (rt.threads + 63) / 64 * 64;
    size_t lds = row_tile_lds(rt.S, units, pad);
    // with N_v = 12 and one RHS per thread each direction's links are staged in LDS too: N_c^2
    // entries per site after the row tile
    const size_t lds_ll = lds + (static_cast<size_t>(rt.S) * NC * NC * sizeof(typename P::G) + 15) / 16 * 16;
    const bool ll = a.nv == 12 && RB == 1 && lds_ll <= kRowLdsCap && lds_ll <= max_lds_per_block();
    const dim3 grid(static_cast<unsigned>(grid_blocks_x8(rt.ntiles, 1)));
    using R = typename P::R;
    const R diag = static_cast<R>(4.0 + a.mass);
    auto U = static_cast<const typename P::G*>(a.gauge);
    auto in = static_cast<const S*>(a.in);
    auto out = static_cast<S*>(a.out);
    auto clov = static_cast<const R*>(a.clover);
    bool ok = true;
    auto go = [&](auto kern) {
        static const bool allowed = allow_lds(kern, kRowLdsCap);
        if (!allowed && lds > 64 * 1024) {
            ok = false;
            return;
        }
        hipLaunchKernelGGL(kern, grid, dim3(block), lds, st, U, in, out, diag, a.g, a.nv, rt, clov, a.epi);
    };
    // the clover term is a separate instantiation: its registers would otherwise lower the occupancy
    // of the plain kernel
    auto pick = [&](auto clov_c) {
        constexpr bool CL = decltype(clov_c)::value;
        if constexpr (RB == 1) {
            if (ll) {  // links staged in LDS with the rows, RHS stride fixed at 12
                lds = lds_ll;
                if (a.dagger)
                    go(wilson_rows_kernel<NC, RB, true, P, 12, true, CL>);
                else
                    go(wilson_rows_kernel<NC, RB, false, P, 12, true, CL>);
                return;
            }
        }
        // runtime RHS stride, links loaded by every thread
        if (a.dagger)
            go(wilson_rows_kernel<NC, RB, true, P, 0, false, CL>);
        else
            go(wilson_rows_kernel<NC, RB, false, P, 0, false, CL>);
    };
    if (clov)
        pick(std::true_type{});
    else
        pick(std::false_type{});
    return ok;
}

// false: an epilogue was asked for and only the direct kernel could take this shape (nothing launched)
template <int NC, int RB, class P>
bool launch_rb(const StencilArgs& a, hipStream_t st) {
    using R = typename P::R;
    if (a.variant == 4 && launch_rows<NC, RB, P>(a, st)) return true;
    if (a.epi.mode != 0) return false;
    // direct loads (selected, or the row tile does not fit this shape)
    const int block = 256;
    const int64_t threads = a.g.vol * (a.nv / RB);
    const dim3 grid(static_cast<unsigned>(grid_blocks_x8(threads, block)));
    const R diag = static_cast<R>(4.0 + a.mass);
    auto U = static_cast<const typename P::G*>(a.gauge);
    auto in = static_cast<const typename P::S*>(a.in);
    auto out = static_cast<typename P::S*>(a.out);
    auto clov = static_cast<const R*>(a.clover);
    const SiteOrder ord = make_site_order(a.g);
    if (a.dagger)
        hipLaunchKernelGGL((wilson_kernel<NC, RB, true, P>), grid, dim3(block), 0, st, U, in, out, diag, a.g, a.nv, ord,
                           clov);
    else
        hipLaunchKernelGGL((wilson_kernel<NC, RB, false, P>), grid, dim3(block), 0, st, U, in, out, diag, a.g, a.nv,
                           ord, clov);
    return true;
}

template <int NC, class P>
bool launch_nc(const StencilArgs& a, hipStream_t st) {
    return a.rb == 2 ? launch_rb<NC, 2, P>(a, st) : launch_rb<NC, 1, P>(a, st);
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

int launch_wilson(const StencilArgs& a, hipStream_t st) {
    switch (a.prec) {
        case DIRAC_FP64: return launch_prec<PrecF64>(a, st);
        case DIRAC_FP32: return launch_prec<PrecF32>(a, st);
        case DIRAC_BF16: return launch_prec<PrecBF16>(a, st);
    }
    return DIRAC_EINVAL;
}

}  // namespace dirac
