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
#include "common.h"
#include "kernels.h"

namespace dirac {

namespace {

__constant__ double c_rho[5] = {0.0, 64.0 / 432.0, 16.0 / 432.0, 4.0 / 432.0, 1.0 / 432.0};
__constant__ double c_halflam[5] = {-120.0 / 64.0, 4.0 / 64.0, 2.0 / 64.0, 1.0 / 64.0, 0.5 / 64.0};

// ---------------------------------------------------------------------------
// Link construction: one thread per (stored direction, site); direction is the slow
// index so that a wavefront shares one direction (uniform loop counts).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool next_perm(int* a, int k) {
    int i = k - 2;
    while (i >= 0 && a[i] >= a[i + 1]) --i;
    if (i < 0) return false;
    int j = k - 1;
    while (a[j] <= a[i]) --j;
    int t = a[i];
    a[i] = a[j];
    a[j] = t;
    for (int l = i + 1, r = k - 1; l < r; ++l, --r) {
        t = a[l];
        a[l] = a[r];
        a[r] = t;
    }
    return true;
}

template <int NC, typename GI, typename GO>
__global__ __launch_bounds__(256) void links_kernel(const GI* __restrict__ U, GO* __restrict__ W, Geom g) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= 40 * g.vol) return;
    const int dir = static_cast<int>(gid / g.vol);
    const int64_t site = gid - static_cast<int64_t>(dir) * g.vol;
    const int d[4] = {dir % 3 - 1, (dir / 3) % 3 - 1, (dir / 9) % 3 - 1, dir / 27 - 1};
    int smu[4], ssg[4], k = 0;
    for (int mu = 0; mu < 4; ++mu)
        if (d[mu] != 0) {
            smu[k] = mu;
            ssg[k] = d[mu];
            ++k;
        }
    const Coord c0 = site_coord(site, g);
    const int ext[4] = {g.nx, g.ny, g.nz, g.nt};

    cx<double> acc[NC][NC];
    for (int a = 0; a < NC; ++a)
        for (int b = 0; b < NC; ++b) acc[a][b] = {0.0, 0.0};
    int perm[4] = {0, 1, 2, 3};
    int npaths = 0;
    do {
        int x[4] = {c0.x, c0.y, c0.z, c0.t};
        cx<double> p[NC][NC];
        for (int a = 0; a < NC; ++a)
            for (int b = 0; b < NC; ++b) p[a][b] = {a == b ? 1.0 : 0.0, 0.0};
        for (int j = 0; j < k; ++j) {
            const int mu = smu[perm[j]];
            const int sg = ssg[perm[j]];
            cx<double> l[NC][NC];
            if (sg > 0) {
                const GI* lp = U + (site_index(x[0], x[1], x[2], x[3], g) * 4 + mu) * NC * NC;
                for (int a = 0; a < NC; ++a)
                    for (int b = 0; b < NC; ++b) l[a][b] = io<double, GI>::ld(lp + a * NC + b);
                x[mu] = wrap(x[mu] + 1, ext[mu]);
            } else {
                x[mu] = wrap(x[mu] - 1, ext[mu]);
                const GI* lp = U + (site_index(x[0], x[1], x[2], x[3], g) * 4 + mu) * NC * NC;
                for (int a = 0; a < NC; ++a)
                    for (int b = 0; b < NC; ++b) l[b][a] = cconj(io<double, GI>::ld(lp + a * NC + b));
            }
            cx<double> q[NC][NC];
            for (int a = 0; a < NC; ++a)
                for (int b = 0; b < NC; ++b) {
                    cx<double> s{0.0, 0.0};
                    for (int e = 0; e < NC; ++e) cfma(s, p[a][e], l[e][b]);
                    q[a][b] = s;
                }
            for (int a = 0; a < NC; ++a)
                for (int b = 0; b < NC; ++b) p[a][b] = q[a][b];
        }
        for (int a = 0; a < NC; ++a)
            for (int b = 0; b < NC; ++b) acc[a][b] = cadd(acc[a][b], p[a][b]);
        ++npaths;
    } while (next_perm(perm, k));
    const double inv = 1.0 / npaths;
    GO* out = W + (site * 40 + dir) * NC * NC;
    for (int a = 0; a < NC; ++a)
        for (int b = 0; b < NC; ++b) io<double, GO>::st(out + a * NC + b, cscale(inv, acc[a][b]));
}

// ---------------------------------------------------------------------------
// Apply: one thread per (site, RB right-hand sides); the 80 directions are a runtime loop
// with wave-uniform direction data.
// ---------------------------------------------------------------------------
template <int NC, int RB, bool DAG, class P>
__global__ __launch_bounds__(256) void brillouin_kernel(const typename P::G* __restrict__ W,
                                                         const typename P::S* __restrict__ in,
                                                         typename P::S* __restrict__ out, typename P::R diag, Geom g,
                                                         int nv, SiteOrder order) {
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
        const R rho = static_cast<R>(DAG ? -c_rho[kh] : c_rho[kh]);
        const R q1 = rho * (ix - 1), q2 = rho * (iy - 1), q3 = rho * (iz - 1), q4 = rho * (it - 1);
        const R lh = static_cast<R>(c_halflam[kh]);
        const int64_t nb = site + (ox[ix] + oy[iy] + oz[iz] + ot[it]);
        const R bsign = sgn_t[it];

        cx<R> l[NC][NC];
        if (dir < 40) {
            const typename P::G* lp = W + (site * 40 + dir) * NC * NC;
#pragma unroll
            for (int a = 0; a < NC; ++a)
#pragma unroll
                for (int b = 0; b < NC; ++b) l[a][b] = cscale(bsign, io<R, typename P::G>::ld(lp + a * NC + b));
        } else {
            const typename P::G* lp = W + (nb * 40 + (80 - dir)) * NC * NC;
#pragma unroll
            for (int a = 0; a < NC; ++a)
#pragma unroll
                for (int b = 0; b < NC; ++b) l[b][a] = cscale(bsign, cconj(io<R, typename P::G>::ld(lp + a * NC + b)));
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
                cx<R>* o = acc[k][a];
                // -lambda_k/2 (spin diagonal)
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    o[s].re -= lh * ch[s].re;
                    o[s].im -= lh * ch[s].im;
                }
                // rho_k sum_mu d_mu g_mu in the chiral basis, one displacement component at a time:
                //   g_4: rows (0,1,2,3) <- (2,3,0,1)
                //   g_3: rows <- (-i 2, +i 3, +i 0, -i 1)
                //   g_2: rows <- (-3, +2, +1, -0)
                //   g_1: rows <- (-i 3, -i 2, +i 1, +i 0)
                if (it != 1) {
                    o[0].re += q4 * ch[2].re; o[0].im += q4 * ch[2].im;
                    o[1].re += q4 * ch[3].re; o[1].im += q4 * ch[3].im;
                    o[2].re += q4 * ch[0].re; o[2].im += q4 * ch[0].im;
                    o[3].re += q4 * ch[1].re; o[3].im += q4 * ch[1].im;
                }
                if (iz != 1) {
                    o[0].re += q3 * ch[2].im; o[0].im -= q3 * ch[2].re;
                    o[1].re -= q3 * ch[3].im; o[1].im += q3 * ch[3].re;
                    o[2].re -= q3 * ch[0].im; o[2].im += q3 * ch[0].re;
                    o[3].re += q3 * ch[1].im; o[3].im -= q3 * ch[1].re;
                }
                if (iy != 1) {
                    o[0].re -= q2 * ch[3].re; o[0].im -= q2 * ch[3].im;
                    o[1].re += q2 * ch[2].re; o[1].im += q2 * ch[2].im;
                    o[2].re += q2 * ch[1].re; o[2].im += q2 * ch[1].im;
                    o[3].re -= q2 * ch[0].re; o[3].im -= q2 * ch[0].im;
                }
                if (ix != 1) {
                    o[0].re += q1 * ch[3].im; o[0].im -= q1 * ch[3].re;
                    o[1].re += q1 * ch[2].im; o[1].im -= q1 * ch[2].re;
                    o[2].re -= q1 * ch[1].im; o[2].im += q1 * ch[1].re;
                    o[3].re -= q1 * ch[0].im; o[3].im += q1 * ch[0].re;
                }
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

template <int NC, int RB, class P>
void launch_rb(const StencilArgs& a, hipStream_t st) {
    using R = typename P::R;
    const int block = 256;
    const int64_t threads = a.g.vol * (a.nv / RB);
    const dim3 grid(static_cast<unsigned>(grid_blocks_x8(threads, block)));
    const R diag = static_cast<R>(a.mass + 120.0 / 64.0);
    auto W = static_cast<const typename P::G*>(a.gauge);
    auto in = static_cast<const typename P::S*>(a.in);
    auto out = static_cast<typename P::S*>(a.out);
    if (a.dagger)
        hipLaunchKernelGGL((brillouin_kernel<NC, RB, true, P>), grid, dim3(block), 0, st, W, in, out, diag, a.g, a.nv,
                           make_site_order(a.g));
    else
        hipLaunchKernelGGL((brillouin_kernel<NC, RB, false, P>), grid, dim3(block), 0, st, W, in, out, diag, a.g,
                           a.nv, make_site_order(a.g));
}

template <int NC, class P>
void launch_nc(const StencilArgs& a, hipStream_t st) {
    switch (a.rb) {
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

template <int NC>
void launch_links_nc(dirac_prec prec, const Geom& g, const void* U, void* W, hipStream_t st) {
    const int block = 256;
    const dim3 grid(static_cast<unsigned>((40 * g.vol + block - 1) / block));
    if (prec == DIRAC_FP64)
        hipLaunchKernelGGL((links_kernel<NC, double2, double2>), grid, dim3(block), 0, st,
                           static_cast<const double2*>(U), static_cast<double2*>(W), g);
    else
        hipLaunchKernelGGL((links_kernel<NC, float2, float2>), grid, dim3(block), 0, st, static_cast<const float2*>(U),
                           static_cast<float2*>(W), g);
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
