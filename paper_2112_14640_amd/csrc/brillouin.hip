// Brillouin operator (Sec. 6): hypercube links W and the 81-point apply.
//
// Directions d in {-1,0,1}^4 are numbered dir = 27(d_t+1) + 9(d_z+1) + 3(d_y+1) + (d_x+1);
// dir = 40 is the centre.  The 40 directions dir < 40 are stored; W_d(n) for dir > 40 is
// W_{-d}(n+d)^+ (Tab. off-axis), read from the neighbour's direction 80 - dir.
//
// Links: W_d(n) is the plain average over the |d|! orderings of the unit steps of d of the
// ordered products of V along each path (a step -mu from x uses V_mu(x-mu)^+).
//
// Apply, with k = |d| (non-zero components), rho = (64,16,4,1)/432, lambda = (-240,8,4,2,1)/64:
//   (D_B u)(n) = (m - lambda_0/2) u(n) + sum_{d != 0} [(rho_k sum_mu d_mu g_mu - lambda_k/2) x W_d(n)] u(n+d)
// which is Eq. app_bril with the derivative factor of Eq. def_ider written out; the adjoint
// negates the rho part (g_5-hermiticity).  In the chiral basis sum_mu c_mu g_mu is
// [[0, B], [B^+, 0]] with B = [[c4 - i c3, -c2 - i c1], [c2 - i c1, c4 + i c3]] (App. C).
// The optional clover term C of Eq. def_clov is added at the centre (hermitian: the adjoint adds it
// unchanged).  With the flag lap the same kernels apply the Brillouin Laplacian of Eq. app_blap,
//   (-1/2 Delta^bri + m^2/2) u(n) = (m^2/2 - lambda_0/2) u(n) - sum_{d != 0} (lambda_|d|/2) W_d(n) u(n+d),
// the spin-trivial part of the stencil (the rho terms are skipped; the caller passes the diagonal).
#include <mutex>
#include <type_traits>

#include "clover.h"
#include "common.h"
#include "kernels.h"
#include "tile.h"

namespace dirac {

namespace {

__constant__ double c_rho[5] = {0.0, 64.0 / 432.0, 16.0 / 432.0, 4.0 / 432.0, 1.0 / 432.0};
__constant__ double c_halflam[5] = {-120.0 / 64.0, 4.0 / 64.0, 2.0 / 64.0, 1.0 / 64.0, 0.5 / 64.0};

// Spin-factor scalars per direction, filled once per device from the two tables above:
// c_spin<R>[dag][flip][dir] = {lambda_k / 2, q_1..q_4} with q_mu = rho_k d_mu (negated for the adjoint)
// and all five negated when flip = 1 (the fermion sign of a t-wrapping hop).  Wave-uniform, so the
// row kernel reads them with scalar loads instead of recomputing them in every lane.
constexpr int kSpinVals = 5;
__constant__ float c_spin_f[2][2][81][kSpinVals];
__constant__ double c_spin_d[2][2][81][kSpinVals];

template <typename R>
__device__ __forceinline__ const R* spin_table(int dag, int flip, int dir);
template <>
__device__ __forceinline__ const float* spin_table<float>(int dag, int flip, int dir) {
    return c_spin_f[dag][flip][dir];
}
template <>
__device__ __forceinline__ const double* spin_table<double>(int dag, int flip, int dir) {
    return c_spin_d[dag][flip][dir];
}

// ---------------------------------------------------------------------------
// Link construction, level by level.  Grouping the |d|! orderings of the unit steps of d by
// their last step gives
//     W_d(n) = (1/|d|) sum_{mu: d_mu != 0} W_{d - s e_mu}(n) L,   s = d_mu,
// with L = V_mu(n + d - e_mu) for s = +1 and L = V_mu(n + d)^+ for s = -1: the average at
// |d| is built from the averages at |d| - 1 of the same site, so a site needs 176 products
// (levels 2, 3 in all 56 directions and the 8 stored ones of level 4) instead of the 1108 of
// the separate paths.  A work-group takes S consecutive sites, holds the levels of its
// sites in LDS (slot = direction number; in the output precision, products accumulated in
// FP64), and writes each site's 40 stored directions as one contiguous block.
// ---------------------------------------------------------------------------
struct LevelDirs {
    unsigned char dir[64];  // level 2 (24 directions), level 3 (32), level 4 stored (8)
};
constexpr LevelDirs make_level_dirs() {
    LevelDirs l{};
    int n = 0;
    for (int k = 2; k <= 4; ++k)
        for (int dir = 0; dir < 81; ++dir) {
            int nz = 0;
            for (int mu = 0, q = dir; mu < 4; ++mu, q /= 3) nz += q % 3 != 1;
            if (nz == k && (k < 4 || dir < 40)) l.dir[n++] = static_cast<unsigned char>(dir);
        }
    return l;
}
__constant__ LevelDirs c_levels = make_level_dirs();
constexpr int kLevelStart[3] = {0, 24, 56};
constexpr int kLevelCount[3] = {24, 32, 8};
constexpr int kDirStride[4] = {1, 3, 9, 27};

template <int NC>
constexpr int link_tile_sites() {
    return NC <= 3 ? 4 : 2;  // 4 x 81 x 9 x 16 B = 46.7 KB of LDS for N_c = 3 in FP64, half in FP32
}
constexpr int kLinkThreads = 128;

template <int NC, typename GI, typename GO>
__global__ __launch_bounds__(kLinkThreads) void links_kernel(const GI* __restrict__ U, GO* __restrict__ W, Geom g) {
    constexpr int S = link_tile_sites<NC>();
    constexpr int L = NC * NC;
    using T = std::conditional_t<sizeof(GO) == 8, float, double>;
    __shared__ cx<T> lw[S][81][L];
    const int64_t site0 = logical_block() * S;
    if (site0 >= g.vol) return;
    const int ns = static_cast<int>(g.vol - site0 < S ? g.vol - site0 : S);
    const int tid = threadIdx.x;
    const int ext[4] = {g.nx, g.ny, g.nz, g.nt};
    auto link_at = [&](const int* c, int mu) __attribute__((always_inline)) {
        return U + (site_index(c[0], c[1], c[2], c[3], g) * 4 + mu) * L;
    };
    // level 1: W_{+e_mu}(n) = V_mu(n), W_{-e_mu}(n) = V_mu(n - e_mu)^+
    for (int u = tid; u < ns * 8 * L; u += kLinkThreads) {
        const int s = u / (8 * L), j = (u / L) % 8, e = u % L;
        const int mu = j >> 1, a = e / NC, b = e % NC;
        const Coord c0 = site_coord(site0 + s, g);
        int c[4] = {c0.x, c0.y, c0.z, c0.t};
        if (j & 1) {
            c[mu] = wrap(c[mu] - 1, ext[mu]);
            lw[s][40 - kDirStride[mu]][e] = cconj(io<T, GI>::ld(link_at(c, mu) + b * NC + a));
        } else {
            lw[s][40 + kDirStride[mu]][e] = io<T, GI>::ld(link_at(c, mu) + e);
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int lev = 0; lev < 3; ++lev) {
        const int k = lev + 2, cnt = kLevelCount[lev];
        const double inv = 1.0 / k;
        for (int u = tid; u < ns * cnt; u += kLinkThreads) {
            const int s = u / cnt;
            const int dir = c_levels.dir[kLevelStart[lev] + (u - s * cnt)];
            const Coord c0 = site_coord(site0 + s, g);
            const int n0[4] = {c0.x, c0.y, c0.z, c0.t};
            int d[4];
            for (int mu = 0, q = dir; mu < 4; ++mu, q /= 3) d[mu] = q % 3 - 1;
            // the links of all last steps are loaded before any product, so their latencies overlap
            GI raw[4][L];
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                if (d[mu] == 0) continue;
                int c[4];
#pragma unroll
                for (int nu = 0; nu < 4; ++nu)
                    c[nu] = wrap(n0[nu] + d[nu] - (nu == mu && d[mu] > 0 ? 1 : 0), ext[nu]);
                const GI* lp = link_at(c, mu);
#pragma unroll
                for (int e = 0; e < L; ++e) raw[mu][e] = lp[e];
            }
            cx<double> acc[NC][NC];
#pragma unroll
            for (int a = 0; a < NC; ++a)
#pragma unroll
                for (int b = 0; b < NC; ++b) acc[a][b] = {0.0, 0.0};
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                if (d[mu] == 0) continue;
                const int sg = d[mu];
                const cx<T>* prev = lw[s][dir - sg * kDirStride[mu]];
                cx<double> l[NC][NC];
#pragma unroll
                for (int a = 0; a < NC; ++a)
#pragma unroll
                    for (int b = 0; b < NC; ++b) {
                        const cx<double> v = io<double, GI>::ld(&raw[mu][a * NC + b]);
                        if (sg > 0)
                            l[a][b] = v;
                        else
                            l[b][a] = cconj(v);
                    }
#pragma unroll
                for (int a = 0; a < NC; ++a)
#pragma unroll
                    for (int e = 0; e < NC; ++e) {
                        const cx<double> pv{prev[a * NC + e].re, prev[a * NC + e].im};
#pragma unroll
                        for (int b = 0; b < NC; ++b) cfma(acc[a][b], pv, l[e][b]);
                    }
            }
#pragma unroll
            for (int a = 0; a < NC; ++a)
#pragma unroll
                for (int b = 0; b < NC; ++b) {
                    const cx<double> v = cscale(inv, acc[a][b]);
                    lw[s][dir][a * NC + b] = {static_cast<T>(v.re), static_cast<T>(v.im)};
                }
        }
        __syncthreads();
    }
    // the stored directions 0..39 of the tile's sites are one contiguous block of W
    GO* out = W + site0 * 40 * L;
    for (int u = tid; u < ns * 40 * L; u += kLinkThreads) {
        const int s = u / (40 * L), r = u - s * 40 * L;
        io<T, GO>::st(out + u, lw[s][r / L][r % L]);
    }
}

// ---------------------------------------------------------------------------
// Apply: one thread per (site, RB right-hand sides); the 80 directions are a runtime loop
// with wave-uniform direction data.
// ---------------------------------------------------------------------------
// o[s] += (sum_mu q_mu g_mu - lh) ch[s] in the chiral basis, one displacement component at a time
// (hx..ht: d_x..d_t non-zero; q_mu = rho_k d_mu, already carrying the adjoint's and the boundary's
// signs, as does lh):
//   g_4: rows (0,1,2,3) <- (2,3,0,1)
//   g_3: rows <- (-i 2, +i 3, +i 0, -i 1)
//   g_2: rows <- (-3, +2, +1, -0)
//   g_1: rows <- (-i 3, -i 2, +i 1, +i 0)
// gamma_<mu>_accumulate: one term alone, o[s] += q (g_mu ch)[s].
template <typename R>
__device__ __forceinline__ void gamma_x_accumulate(cx<R> (&o)[4], const cx<R> (&ch)[4], R q1) {
    o[0].re += q1 * ch[3].im; o[0].im -= q1 * ch[3].re;
    o[1].re += q1 * ch[2].im; o[1].im -= q1 * ch[2].re;
    o[2].re -= q1 * ch[1].im; o[2].im += q1 * ch[1].re;
    o[3].re -= q1 * ch[0].im; o[3].im += q1 * ch[0].re;
}
template <typename R>
__device__ __forceinline__ void gamma_y_accumulate(cx<R> (&o)[4], const cx<R> (&ch)[4], R q2) {
    o[0].re -= q2 * ch[3].re; o[0].im -= q2 * ch[3].im;
    o[1].re += q2 * ch[2].re; o[1].im += q2 * ch[2].im;
    o[2].re += q2 * ch[1].re; o[2].im += q2 * ch[1].im;
    o[3].re -= q2 * ch[0].re; o[3].im -= q2 * ch[0].im;
}
template <typename R>
__device__ __forceinline__ void gamma_z_accumulate(cx<R> (&o)[4], const cx<R> (&ch)[4], R q3) {
    o[0].re += q3 * ch[2].im; o[0].im -= q3 * ch[2].re;
    o[1].re -= q3 * ch[3].im; o[1].im += q3 * ch[3].re;
    o[2].re -= q3 * ch[0].im; o[2].im += q3 * ch[0].re;
    o[3].re += q3 * ch[1].im; o[3].im -= q3 * ch[1].re;
}
template <typename R>
__device__ __forceinline__ void gamma_t_accumulate(cx<R> (&o)[4], const cx<R> (&ch)[4], R q4) {
    o[0].re += q4 * ch[2].re; o[0].im += q4 * ch[2].im;
    o[1].re += q4 * ch[3].re; o[1].im += q4 * ch[3].im;
    o[2].re += q4 * ch[0].re; o[2].im += q4 * ch[0].im;
    o[3].re += q4 * ch[1].re; o[3].im += q4 * ch[1].im;
}

template <typename R>
__device__ __forceinline__ void spin_accumulate(cx<R> (&o)[4], const cx<R> (&ch)[4], R lh, R q1, R q2, R q3, R q4,
                                                bool hx, bool hy, bool hz, bool ht) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        o[s].re -= lh * ch[s].re;
        o[s].im -= lh * ch[s].im;
    }
    if (ht) gamma_t_accumulate(o, ch, q4);
    if (hz) gamma_z_accumulate(o, ch, q3);
    if (hy) gamma_y_accumulate(o, ch, q2);
    if (hx) gamma_x_accumulate(o, ch, q1);
}

template <int NC, int RB, bool DAG, class P>
__global__ __launch_bounds__(256) void brillouin_kernel(const typename P::G* __restrict__ W,
                                                         const typename P::S* __restrict__ in,
                                                         typename P::S* __restrict__ out, typename P::R diag, Geom g,
                                                         int nv, SiteOrder order, const typename P::R* __restrict__ clov,
                                                         int lap) {
    using R = typename P::R;
    using S = typename P::S;
    const int nrg = nv / RB;
    const int64_t gid = logical_block() * blockDim.x + threadIdx.x;
    if (gid >= g.vol * nrg) return;
    const int64_t idx = gid / nrg;
    const int r0 = static_cast<int>(gid - idx * nrg) * RB;
    const int64_t site = ordered_site(idx, order, g);
    const Coord c = site_coord(site, g);
    const int64_t vs = static_cast<int64_t>(NC) * 4 * nv;

    cx<R> acc[RB][NC][4];
    const S* centre = in + site * vs + r0;
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[k][a][s] = cscale(diag, io<R, S>::ld(centre + (a * 4 + s) * nv + k));
    if (clov) clover_add<NC, RB>(acc, centre, nv, clov + site * clover_reals<NC>());

    // neighbour offsets along each axis for steps -1, 0, +1 (with the periodic wrap) and the
    // fermion sign of the t steps; per direction the neighbour is site + four offsets
    // (site offsets fit in 32 bits: the library limits the volume to < 2^31 sites)
    const int sy = g.nx, sz = g.nx * g.ny, stt = sz * g.nz;
    const int ox[3] = {c.x == 0 ? g.nx - 1 : -1, 0, c.x == g.nx - 1 ? 1 - g.nx : 1};
    const int oy[3] = {(c.y == 0 ? g.ny - 1 : -1) * sy, 0, (c.y == g.ny - 1 ? 1 - g.ny : 1) * sy};
    const int oz[3] = {(c.z == 0 ? g.nz - 1 : -1) * sz, 0, (c.z == g.nz - 1 ? 1 - g.nz : 1) * sz};
    const int ot[3] = {(c.t == 0 ? g.nt - 1 : -1) * stt, 0, (c.t == g.nt - 1 ? 1 - g.nt : 1) * stt};
    const R sgn_t[3] = {(g.apbc && c.t == 0) ? R(-1) : R(1), R(1), (g.apbc && c.t == g.nt - 1) ? R(-1) : R(1)};

    for (int dir = 0; dir < 81; ++dir) {
        if (dir == 40) continue;
        // wave-uniform direction data
        const int ix = dir % 3, iy = (dir / 3) % 3, iz = (dir / 9) % 3, it = dir / 27;
        const int kh = (ix != 1) + (iy != 1) + (iz != 1) + (it != 1);
        // the fermion sign of a t-wrapping hop rides on the spin factor (five scalars)
        const R bsign = sgn_t[it];
        const R rho = bsign * static_cast<R>(DAG ? -c_rho[kh] : c_rho[kh]);
        const R q1 = rho * (ix - 1), q2 = rho * (iy - 1), q3 = rho * (iz - 1), q4 = rho * (it - 1);
        const R lh = bsign * static_cast<R>(c_halflam[kh]);
        const int64_t nb = site + (ox[ix] + oy[iy] + oz[iz] + ot[it]);

        cx<R> l[NC][NC];
        if (dir < 40) {
            const typename P::G* lp = W + (site * 40 + dir) * NC * NC;
#pragma unroll
            for (int a = 0; a < NC; ++a)
#pragma unroll
                for (int b = 0; b < NC; ++b) l[a][b] = io<R, typename P::G>::ld(lp + a * NC + b);
        } else {
            const typename P::G* lp = W + (nb * 40 + (80 - dir)) * NC * NC;
#pragma unroll
            for (int a = 0; a < NC; ++a)
#pragma unroll
                for (int b = 0; b < NC; ++b) l[b][a] = cconj(io<R, typename P::G>::ld(lp + a * NC + b));
        }
        const S* nbp = in + nb * vs + r0;
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            cx<R> p[NC][4];
#pragma unroll
            for (int b = 0; b < NC; ++b)
#pragma unroll
                for (int s = 0; s < 4; ++s) p[b][s] = io<R, S>::ld(nbp + (b * 4 + s) * nv + k);
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                cx<R> ch[4] = {{R(0), R(0)}, {R(0), R(0)}, {R(0), R(0)}, {R(0), R(0)}};
#pragma unroll
                for (int b = 0; b < NC; ++b)
#pragma unroll
                    for (int s = 0; s < 4; ++s) cfma(ch[s], l[a][b], p[b][s]);
                spin_accumulate(acc[k][a], ch, lh, q1, q2, q3, q4, !lap && ix != 1, !lap && iy != 1, !lap && iz != 1,
                                !lap && it != 1);
            }
        }
    }

    S* o = out + site * vs + r0;
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int s = 0; s < 4; ++s) io<R, S>::st(o + (a * 4 + s) * nv + k, acc[k][a][s]);
}


// Row-tiled apply: a work-group owns one x-row (every RHS) and walks the 27 rows at (y, z, t)
// offsets in {-1,0,1}^3 (row copy rc = 9 (d_t+1) + 3 (d_z+1) + (d_y+1)).  Each such row is copied
// into LDS with contiguous 16-byte loads and serves the three directions d_x = -1, 0, +1
// (periodic within the row).  With it comes a window of three consecutive stored links per
// site of one row: for rc < 13 the directions dir0 .. dir0 + 2 (dir0 = 27 it + 9 iz + 3 iy) of the
// own row; for rc > 13 the directions 78 - dir0 .. 80 - dir0 of the neighbour row, whose adjoints
// are the links of the directions 80 - dir (Tab. off-axis); for rc = 13 direction 39 of the own
// row serves d_x = -1 as stored and d_x = +1 as the adjoint at x + 1.  The window holds each link as
// applied: adjoints transposed and conjugated, and the fermion sign of a t step across the boundary
// folded in, so that every hop is the same plain product.  The next row copy is in flight (in
// registers) while the current one is consumed.  The three hops of a row, whose spin factors share
// their gamma_y..gamma_t terms up to fixed ratios, go into one accumulator (15432 instead of 18648
// multiply-adds per site and RHS with N_c = 3, the App. E count unchanged; the colour-split form
// shares it between the d_x = -1 and +1 hops only).  Three waves per SIMD
// cap the registers at 168 (FP32 and BF16 fit, the segmented forms spill a few values); FP64, whose
// operands take twice the registers, takes the colour-split form (CS) at three waves per SIMD.
template <int NC, int RB, bool DAG, class P, int NVC, bool SEG, bool CS = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(typename P::R) == 8 && !CS ? 2 : 3))) void brillouin_rows_kernel(const typename P::G* __restrict__ W,
                                                             const typename P::S* __restrict__ in,
                                                             typename P::S* __restrict__ out, typename P::R diag,
                                                             Geom g, int nv, RowTile rt,
                                                             const typename P::R* __restrict__ clov, int lap) {
    using R = typename P::R;
    using S = typename P::S;
    using G = typename P::G;
    // CS (colour split): a thread owns one colour row a of one RHS of its site (N_c threads per site and
    // RHS), so its accumulators, link row and share of the row copy are a third as large
    static_assert(RB == 1, "the row form takes one RHS per thread");
    constexpr int PER = CS ? RowUnits<NC, RB, P>::PER / NC : RowUnits<NC, RB, P>::PER;
    constexpr int NA = CS ? 1 : NC;  // colour rows per thread
    constexpr int L = NC * NC;
    extern __shared__ __align__(16) u32x4 rtile[];
    if constexpr (NVC > 0) nv = NVC;

    const int64_t tix = logical_block();
    if (tix >= rt.ntiles) return;
    const uint32_t nseg = static_cast<uint32_t>(rt.nseg);
    const uint32_t rq = static_cast<uint32_t>(tix) / nseg;
    const int x0 = static_cast<int>(static_cast<uint32_t>(tix) - rq * nseg) * rt.S;  // first site of the segment
    const uint32_t rho = tile_row(rq, rt, g);
    const uint32_t tid = threadIdx.x;
    const bool active = tid < static_cast<uint32_t>(rt.threads);
    const uint32_t tt = active ? tid : tid - rt.threads;  // padding threads shadow a real one
    const uint32_t j = fast_div(tt, rt.magic_nrg);      // site within the segment
    const int rg = static_cast<int>(tt - j * rt.nrg);   // CS: ca * nv + rhs
    const int ca = CS ? rg / nv : 0;                    // CS: the thread's colour row
    const int col = CS ? rg - ca * nv : rg * RB;        // first RHS column of the thread
    const int x = x0 + static_cast<int>(j);
    int cy, cz, ct;
    {
        const uint32_t q = rho / static_cast<uint32_t>(g.ny);
        cy = static_cast<int>(rho - q * g.ny);
        const uint32_t q2 = q / static_cast<uint32_t>(g.nz);
        cz = static_cast<int>(q - q2 * g.nz);
        ct = static_cast<int>(q2);
    }
    const int64_t own_start = static_cast<int64_t>(rho) * g.nx;
    const u32x4* src = reinterpret_cast<const u32x4*>(in);
    // LDS: with SEG, copy site c = 0 .. S + 1 holds x = x0 - 1 + c (periodic); without, the whole row
    // (c = x, S = n_x, neighbours wrap inside it).  Then the link window.
    constexpr int OFF = SEG ? 1 : 0;  // copy site of the segment's first site
    const int SC = rt.S + 2 * OFF;    // sites per copy
    // the link window, slot-major: lwin[slot][copy site][L], slot = one of the three stored directions
    const uint32_t PADU = row_pad(rt.units, static_cast<uint32_t>(nv) * static_cast<uint32_t>(sizeof(S)) / 4u);
    const uint32_t SU = rt.units + PADU;  // units per site of the row copy
    G* lwin = reinterpret_cast<G*>(rtile + SC * SU);
    const uint32_t WS = static_cast<uint32_t>(SC) * L;  // elements per slot
    // Each load instruction of the window covers one slot: KPS loads per slot, each lane taking entry
    // q * threads + tt of it (checked at launch: SC * L <= KPS * threads); lanes past the slot repeat its
    // last entry and store nothing.  The slot's transposition, sign and scale are then wave-uniform.
    constexpr int KPS = NC >= 4 ? 2 : 1;
    constexpr int PERL = 3 * KPS;
    uint32_t woff[KPS], wofft[KPS];  // the lane's element in a stored direction block: as stored, transposed
#pragma unroll
    for (int q = 0; q < KPS; ++q) {
        const uint32_t e = min(q * static_cast<uint32_t>(rt.threads) + tt, WS - 1u);
        const uint32_t sx = e / L, ab = e - sx * L;
        const uint32_t xs = SEG ? static_cast<uint32_t>(wrap(x0 - 1 + static_cast<int>(sx), g.nx)) : sx;
        woff[q] = xs * 40u * L + ab;
        wofft[q] = xs * 40u * L + (ab % NC) * NC + ab / NC;
    }
    uint32_t slot[PER];      // main units: the S sites of the segment, copy sites 1 .. S
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const uint32_t u = k * static_cast<uint32_t>(rt.threads) + tt;
        slot[k] = u + fast_div(u, rt.magic_units) * PADU + OFF * SU;
    }
    // halo units h = tt and tt + threads (< 2 units) copy the sites x0 - 1 (copy site 0) and x0 + S
    // (copy site S + 1)
    bool halo[2];
    uint32_t hslot[2];
    uint32_t hsrc[2];  // unit index relative to the start of the copied row
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const uint32_t h = tt + q * static_cast<uint32_t>(rt.threads);
        halo[q] = SEG && h < 2u * rt.units;
        const uint32_t hs = h < static_cast<uint32_t>(rt.units) ? 0u : 1u;
        const uint32_t hcu = h - hs * rt.units;
        hslot[q] = (hs ? rt.S + 1 : 0) * SU + hcu;
        hsrc[q] = static_cast<uint32_t>(hs ? wrap(x0 + rt.S, g.nx) : wrap(x0 - 1, g.nx)) * rt.units + hcu;
    }
    auto row_start = [&](int rc) __attribute__((always_inline)) {
        const int dy = rc % 3 - 1, dz = (rc / 3) % 3 - 1, dt = rc / 9 - 1;
        const int y = wrap(cy + dy, g.ny), z = wrap(cz + dz, g.nz), t = wrap(ct + dt, g.nt);
        return ((static_cast<int64_t>(t) * g.nz + z) * g.ny + y) * g.nx;
    };
    u32x4 pre[PER];
    u32x4 hpre[2];
    G lpre[PERL];
    // row copies and link windows are buffer loads over one lattice row: a scalar base per row, 32-bit
    // offsets per lane (a read past the row returns zero instead of touching memory)
    const uint32_t row_bytes = static_cast<uint32_t>(g.nx) * rt.units * 16u;
    const uint32_t wrow_bytes = static_cast<uint32_t>(g.nx) * 40u * L * static_cast<uint32_t>(sizeof(G));
    auto fetch = [&](int rc) __attribute__((always_inline)) {
        const int64_t start = row_start(rc);
        const auto rrow = raw_buffer(src + start * rt.units, row_bytes);
#pragma unroll
        for (int k = 0; k < PER; ++k)
            pre[k] = buffer_load_unit<u32x4>(rrow, tt * 16u,
                                             (static_cast<uint32_t>(x0) * rt.units + k * static_cast<uint32_t>(rt.threads)) *
                                                 16u);
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (SEG && halo[q]) hpre[q] = buffer_load_unit<u32x4>(rrow, hsrc[q] * 16u, 0u);
        const int dir0 = 9 * (3 * (rc / 9) + (rc / 3) % 3) + 3 * (rc % 3);
        const int64_t lstart = rc <= 13 ? own_start : start;
        const int wb = rc < 13 ? dir0 : (rc == 13 ? 37 : 78 - dir0);
        const auto rw = raw_buffer(W + lstart * 40 * L, wrow_bytes);
        // window slot ws holds W_d(n) as applied: for rc > 13 every slot is the adjoint of the stored
        // link (element (a, b) <- conj of stored (b, a)); for rc = 13 slot 2 holds direction 39 as stored
        // and slot 0 its adjoint
#pragma unroll
        for (int k = 0; k < PERL; ++k) {
            const int ws = k / KPS, q = k % KPS;
            const bool adj = rc > 13 || (rc == 13 && ws == 0);
            const uint32_t from = (adj ? wofft[q] : woff[q]) +
                                  static_cast<uint32_t>(wb + (rc == 13 && ws == 0 ? 2 : ws)) * L;
            lpre[k] = buffer_load_unit<G>(rw, from * static_cast<uint32_t>(sizeof(G)), 0u);
        }
    };
    auto at = [&](int c) __attribute__((always_inline)) {
        return reinterpret_cast<const S*>(rtile + c * SU) + col;
    };

    cx<R> acc[RB][NA][4];
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[k][a][s] = {R(0), R(0)};

    fetch(0);
    for (int rc = 0; rc < 27; ++rc) {
        __syncthreads();  // the previous row copy has been consumed
#pragma unroll
        for (int k = 0; k < PER; ++k) rtile[slot[k]] = pre[k];
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (SEG && halo[q]) rtile[hslot[q]] = hpre[q];
        // The window as applied: the adjoint's conjugation, the fermion sign of a t step across the boundary
        // (all three hops of a row take the same t step) and, for the three-hop accumulation below, the
        // d_x = 0 hop times 4 (slot 1 outside the centre row) are factors of the real and imaginary parts,
        // uniform per slot.  They are taken from a copy of rc made opaque here, after the barrier: taken at
        // the loads, they would make the compiler wait for the prefetch there.
        {
            int rs = rc;
            asm volatile("" : "+s"(rs));
            const int its = rs / 9;
            const bool bflip = g.apbc && ((its == 0 && ct == 0) || (its == 2 && ct == g.nt - 1));
#pragma unroll
            for (int k = 0; k < PERL; ++k) {
                const int ws = k / KPS, q = k % KPS;
                const bool adj = rs > 13 || (rs == 13 && ws == 0);
                const R sc = (!CS && ws == 1 && rs != 13) ? R(4) : R(1);
                const R fx = bflip ? -sc : sc;
                const R fy = adj != bflip ? -sc : sc;
                const uint32_t u = q * static_cast<uint32_t>(rt.threads) + tt;
                if (u < WS) {
                    G v = lpre[k];
                    v.x *= fx;
                    v.y *= fy;
                    lwin[ws * WS + u] = v;
                }
            }
        }
        __syncthreads();
        // the last pass refetches its own row (a cache hit): an unconditional fetch keeps the prefetched
        // values in the registers they are loaded into
        fetch(rc < 26 ? rc + 1 : 26);
        if (active) {
            const int iy = rc % 3, iz = (rc / 3) % 3, it = rc / 9;
            const int dir0 = 27 * it + 9 * iz + 3 * iy;  // + ix for d_x = ix - 1
            const bool hy = !lap && iy != 1, hz = !lap && iz != 1, ht = !lap && it != 1;
            // The link W_d(n) of the hop d_x = ix - 1, as applied, and the copy site of its neighbour: for
            // rc < 13 (and rc = 13 with d_x = -1) W_d is stored at the own site, else it is the adjoint of the
            // link stored at n + d, which the window already holds transposed and conjugated (CS: only the
            // thread's row ca of W_d)
            auto hop_link = [&](int ix, cx<R> (&l)[NA][NC]) __attribute__((always_inline)) {
                const int cn = SEG ? static_cast<int>(j) + ix : wrap(static_cast<int>(j) + ix - 1, g.nx);
                const bool adj = rc > 13 || (rc == 13 && ix == 2);
                const G* lp = lwin + (rc < 13 ? ix : (rc == 13 ? (ix == 2 ? 0 : 2) : 2 - ix)) * WS +
                              (adj ? cn : static_cast<int>(j) + OFF) * L;
#pragma unroll
                for (int a = 0; a < NA; ++a)
#pragma unroll
                    for (int b = 0; b < NC; ++b) l[a][b] = io<R, G>::ld(lp + ((CS ? ca : a) * NC + b));
                return cn;
            };
            // c[a] += (W_d u(n + d))_a, one neighbour colour at a time
            auto hop_add = [&](int ix, cx<R> (&c)[NA][4]) __attribute__((always_inline)) {
                cx<R> l[NA][NC];
                const S* nbp = at(hop_link(ix, l));
#pragma unroll
                for (int b = 0; b < NC; ++b) {
                    cx<R> pb[4];
#pragma unroll
                    for (int s = 0; s < 4; ++s) pb[s] = io<R, S>::ld(nbp + (b * 4 + s) * nv);
#pragma unroll
                    for (int a = 0; a < NA; ++a)
#pragma unroll
                        for (int s = 0; s < 4; ++s) cfma(c[a][s], l[a][b], pb[s]);
                }
            };
            if (rc == 13) {  // d_x = 0 is the centre: (m - lambda_0 / 2) u(n), plus the clover term
                const S* nbp = at(static_cast<int>(j) + OFF);
#pragma unroll
                for (int a = 0; a < NA; ++a)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const cx<R> v = io<R, S>::ld(nbp + ((CS ? ca : a) * 4 + s) * nv);
                        acc[0][a][s].re += diag * v.re;
                        acc[0][a][s].im += diag * v.im;
                    }
                if constexpr (!CS)  // the launcher takes the colour-split form only without a clover field
                    if (clov) clover_add<NC, RB>(acc, nbp, nv, clov + (own_start + x) * clover_reals<NC>());
            }
            const R* sm = spin_table<R>(DAG ? 1 : 0, 0, dir0);
            const R* sp = spin_table<R>(DAG ? 1 : 0, 0, dir0 + 2);
            if constexpr (CS) {
                // the colour-split form runs fastest with the d_x = 0 hop on its own and the d_x = -1, +1
                // hops sharing one accumulator: S_- chi_- + S_+ chi_+ = S_+ (chi_- + chi_+) + 2 q_- gamma_x chi_-
                if (rc != 13) {
                    const R* sv = spin_table<R>(DAG ? 1 : 0, 0, dir0 + 1);
                    cx<R> c0[NA][4] = {};
                    hop_add(1, c0);
#pragma unroll
                    for (int a = 0; a < NA; ++a)
                        spin_accumulate(acc[0][a], c0[a], sv[0], sv[1], sv[2], sv[3], sv[4], false, hy, hz, ht);
                }
                cx<R> c[NA][4] = {};
                hop_add(0, c);
                if (!lap) {
#pragma unroll
                    for (int a = 0; a < NA; ++a) gamma_x_accumulate(acc[0][a], c[a], R(2) * sm[1]);
                }
                hop_add(2, c);
#pragma unroll
                for (int a = 0; a < NA; ++a)
                    spin_accumulate(acc[0][a], c[a], sp[0], sp[1], sp[2], sp[3], sp[4], !lap, hy, hz, ht);
            } else {
                // The three hops of a row share one accumulator c.  With k the number of non-zero components of
                // d_x = +-1 (and k - 1 for d_x = 0), S_pm = -l + R pm q gamma_x with l = lambda_k / 2 and
                // R = sum over y, z, t of rho_k d_mu gamma_mu; the d_x = 0 hop has S_0 = -2 l + 4 R (rho and
                // lambda fall by 4 and 2 per unit of k).  So S_- chi_- + S_+ chi_+ + S_0 chi_0 =
                //   2 q_- gamma_x chi_- + (q_+ gamma_x - l / 2) (chi_- + chi_+) + (R - l / 2) (chi_- + chi_+ + 4 chi_0),
                // taken as c = chi_-, then c += chi_+, then c += 4 chi_0 (its link is stored times 4).  In the
                // centre row the last step is -l / 2 alone.
                const R lq = R(0.5) * sp[0];
                cx<R> c[NA][4] = {};
                hop_add(0, c);
                if (!lap) {
#pragma unroll
                    for (int a = 0; a < NA; ++a) gamma_x_accumulate(acc[0][a], c[a], R(2) * sm[1]);
                }
                hop_add(2, c);
#pragma unroll
                for (int a = 0; a < NA; ++a)
                    spin_accumulate(acc[0][a], c[a], lq, sp[1], sp[2], sp[3], sp[4], !lap, false, false, false);
                if (rc != 13) hop_add(1, c);
#pragma unroll
                for (int a = 0; a < NA; ++a)
                    spin_accumulate(acc[0][a], c[a], lq, sp[1], sp[2], sp[3], sp[4], false, hy, hz, ht);
            }
        }
    }
    __syncthreads();
    if (active) {
        S* o = const_cast<S*>(at(static_cast<int>(j) + OFF));
#pragma unroll
        for (int k = 0; k < RB; ++k)
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int s = 0; s < 4; ++s) io<R, S>::st(o + ((CS ? ca : a) * 4 + s) * nv + k, acc[k][a][s]);
    }
    __syncthreads();
    u32x4* dst = reinterpret_cast<u32x4*>(out) + (own_start + x0) * rt.units;
    const uint32_t total = static_cast<uint32_t>(rt.S) * rt.units;
    for (uint32_t u = tid; u < total; u += blockDim.x) dst[u] = rtile[u + fast_div(u, rt.magic_units) * PADU + OFF * SU];
}


// Fill c_spin_f / c_spin_d on the current device (once per device, thread-safe).  false on failure.
bool ensure_spin_table() {
    static std::mutex mu;
    static bool done[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
    std::lock_guard<std::mutex> lock(mu);
    if (done[dev]) return true;
    const double rho[5] = {0.0, 64.0 / 432.0, 16.0 / 432.0, 4.0 / 432.0, 1.0 / 432.0};
    const double halflam[5] = {-120.0 / 64.0, 4.0 / 64.0, 2.0 / 64.0, 1.0 / 64.0, 0.5 / 64.0};
    static double td[2][2][81][kSpinVals];
    static float tf[2][2][81][kSpinVals];
    for (int dag = 0; dag < 2; ++dag)
        for (int flip = 0; flip < 2; ++flip)
            for (int dir = 0; dir < 81; ++dir) {
                const int d[4] = {dir % 3 - 1, (dir / 3) % 3 - 1, (dir / 9) % 3 - 1, dir / 27 - 1};
                const int k = (d[0] != 0) + (d[1] != 0) + (d[2] != 0) + (d[3] != 0);
                const double sg = flip ? -1.0 : 1.0;
                const double r = sg * (dag ? -rho[k] : rho[k]);
                td[dag][flip][dir][0] = sg * halflam[k];
                for (int mu = 0; mu < 4; ++mu) td[dag][flip][dir][1 + mu] = r * d[mu];
                for (int v = 0; v < kSpinVals; ++v) tf[dag][flip][dir][v] = static_cast<float>(td[dag][flip][dir][v]);
            }
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_spin_d), td, sizeof(td)) != hipSuccess) return false;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_spin_f), tf, sizeof(tf)) != hipSuccess) return false;
    done[dev] = true;
    return true;
}

// The centre coefficient: m - lambda_0/2 for D_B, m^2/2 - lambda_0/2 for the Laplacian.
double centre_coefficient(const StencilArgs& a) {
    return (a.laplace ? 0.5 * a.mass * a.mass : a.mass) + 120.0 / 64.0;
}

template <int NC, int RB, class P>
bool launch_rows(const StencilArgs& a, hipStream_t st) {
    using S = typename P::S;
    using R = typename P::R;
    const size_t block_bytes = static_cast<size_t>(NC) * 4 * a.nv * sizeof(S);
    if (block_bytes % 16 != 0 || !tile_aligned(a)) return false;
    const int units = static_cast<int>(block_bytes / 16);
    // FP64: one thread per (site, RHS) where its two waves per SIMD hold the registers (N_c <= 3, a few
    // spills at N_c = 3), else the colour-split form (one colour row of one RHS per thread, three waves
    // per SIMD), which carries no clover term (that case keeps the direct kernel)
    constexpr bool kFP64 = sizeof(R) == 8;
    const int64_t rows = a.g.vol / a.g.nx;
    // segment: the largest divisor of n_x with at most 256 threads (at most 512 if none), at least
    // 64 threads and enough threads for the two halo sites (two units each) and the link window
    auto plan = [&](bool cs, int& seg, size_t& lds) {
        const int nrg = cs ? a.nv * NC : a.nv / RB;
        auto fits = [&](int d, int cap) {
            const int64_t th = static_cast<int64_t>(d) * nrg;
            return a.g.nx % d == 0 && th <= cap && th >= 64 && units <= th &&
                   static_cast<int64_t>(d + 2) * NC * NC <= (NC >= 4 ? 2 : 1) * th;
        };
        seg = 0;
        for (int cap : {256, 512}) {
            for (int d = a.g.nx; d >= 1 && !seg; --d)
                if (fits(d, cap)) seg = d;
            if (seg) break;
        }
        if (seg == 0) return false;
        const int sc = seg + (seg != a.g.nx ? 2 : 0);  // sites per copy
        lds = static_cast<size_t>(sc) * (units + row_pad(units, a.nv * sizeof(S) / 4)) * 16 +
              static_cast<size_t>(sc) * 3 * NC * NC * sizeof(typename P::G);
        return lds <= 64 * 1024;
    };
    int seg = 0;
    size_t lds = 0;
    bool cs = false;
    if (!kFP64 || NC <= 3) {
        if (!plan(false, seg, lds)) {
            if (!kFP64 || a.clover || RB != 1 || !plan(true, seg, lds)) return false;
            cs = true;
        }
    } else {
        if (a.clover || RB != 1 || !plan(true, seg, lds)) return false;
        cs = true;
    }
    const bool segmented = seg != a.g.nx;
    const int nrg = cs ? a.nv * NC : a.nv / RB;
    if (!ensure_spin_table()) return false;  // the direct kernel needs no table
    RowTile rt{};
    rt.R = 1;
    rt.S = seg;
    rt.nseg = a.g.nx / seg;
    rt.nrg = nrg;
    rt.units = units;
    rt.row_units = a.g.nx * units;
    rt.threads = seg * nrg;
    rt.ntiles = rows * rt.nseg;
    rt.magic_nrg = div_magic(nrg);
    rt.magic_nx = div_magic(a.g.nx);
    rt.magic_units = div_magic(units);
    rt.magic_row_units = div_magic(rt.row_units);
    if (!row_order(4, a.g, rt)) return false;
    const int block = (rt.threads + 63) / 64 * 64;
    const dim3 grid(static_cast<unsigned>(grid_blocks_x8(rt.ntiles, 1)));
    const R diag = static_cast<R>(centre_coefficient(a));
    auto W = static_cast<const typename P::G*>(a.gauge);
    auto in = static_cast<const S*>(a.in);
    auto out = static_cast<S*>(a.out);
    auto clov = static_cast<const R*>(a.clover);
    const int lap = a.laplace ? 1 : 0;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(block), lds, st, W, in, out, diag, a.g, a.nv, rt, clov, lap);
    };
    auto pick = [&](auto seg_c, auto cs_c) {
        constexpr bool SG = decltype(seg_c)::value;
        constexpr bool C = decltype(cs_c)::value;
        if (a.nv == 12 && RB == 1) {
            if (a.dagger)
                go(brillouin_rows_kernel<NC, RB, true, P, 12, SG, C>);
            else
                go(brillouin_rows_kernel<NC, RB, false, P, 12, SG, C>);
        } else {
            if (a.dagger)
                go(brillouin_rows_kernel<NC, RB, true, P, 0, SG, C>);
            else
                go(brillouin_rows_kernel<NC, RB, false, P, 0, SG, C>);
        }
    };
    auto pick_seg = [&](auto cs_c) {
        if (segmented)
            pick(std::true_type{}, cs_c);
        else
            pick(std::false_type{}, cs_c);
    };
    if constexpr (kFP64) {
        if (cs) {
            pick_seg(std::true_type{});
            return true;
        }
        if constexpr (NC <= 3) pick_seg(std::false_type{});
    } else {
        pick_seg(std::false_type{});
    }
    return true;
}

template <int NC, int RB, class P>
void launch_rb(const StencilArgs& a, hipStream_t st) {
    using R = typename P::R;
    if (a.variant == 4 && launch_rows<NC, RB, P>(a, st)) return;
    const int block = 256;
    const int64_t threads = a.g.vol * (a.nv / RB);
    const dim3 grid(static_cast<unsigned>(grid_blocks_x8(threads, block)));
    const R diag = static_cast<R>(centre_coefficient(a));
    auto W = static_cast<const typename P::G*>(a.gauge);
    auto in = static_cast<const typename P::S*>(a.in);
    auto out = static_cast<typename P::S*>(a.out);
    auto clov = static_cast<const R*>(a.clover);
    const int lap = a.laplace ? 1 : 0;
    if (a.dagger)
        hipLaunchKernelGGL((brillouin_kernel<NC, RB, true, P>), grid, dim3(block), 0, st, W, in, out, diag, a.g, a.nv,
                           make_site_order(a.g), clov, lap);
    else
        hipLaunchKernelGGL((brillouin_kernel<NC, RB, false, P>), grid, dim3(block), 0, st, W, in, out, diag, a.g,
                           a.nv, make_site_order(a.g), clov, lap);
}

template <int NC, class P>
void launch_nc(const StencilArgs& a, hipStream_t st) {
    launch_rb<NC, 1, P>(a, st);
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

template <int NC>
void launch_links_nc(dirac_prec prec, const Geom& g, const void* U, void* W, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>(grid_blocks_x8(g.vol, link_tile_sites<NC>())));
    if (prec == DIRAC_FP64)
        hipLaunchKernelGGL((links_kernel<NC, double2, double2>), grid, dim3(kLinkThreads), 0, st,
                           static_cast<const double2*>(U), static_cast<double2*>(W), g);
    else
        hipLaunchKernelGGL((links_kernel<NC, float2, float2>), grid, dim3(kLinkThreads), 0, st,
                           static_cast<const float2*>(U), static_cast<float2*>(W), g);
}

}  // namespace

int launch_brillouin(const StencilArgs& a, hipStream_t st) {
    switch (a.prec) {
        case DIRAC_FP64: return launch_prec<PrecF64>(a, st);
        case DIRAC_FP32: return launch_prec<PrecF32>(a, st);
        case DIRAC_BF16: return launch_prec<PrecBF16>(a, st);
    }
    return DIRAC_EINVAL;
}

int launch_brillouin_links(dirac_prec prec, int nc, const Geom& g, const void* U, void* W, hipStream_t st) {
    switch (nc) {
        case 1: launch_links_nc<1>(prec, g, U, W, st); break;
        case 2: launch_links_nc<2>(prec, g, U, W, st); break;
        case 3: launch_links_nc<3>(prec, g, U, W, st); break;
        case 4: launch_links_nc<4>(prec, g, U, W, st); break;
        default: return DIRAC_EUNSUPPORTED;
    }
    return DIRAC_OK;
}

}  // namespace dirac
