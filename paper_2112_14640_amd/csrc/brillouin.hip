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
                                                         int nv) {
    using R = typename P::R;
    using S = typename P::S;
    const int nrg = nv / RB;
    const int64_t gid = logical_block() * blockDim.x + threadIdx.x;
    if (gid >= g.vol * nrg) return;
    const int64_t site = gid / nrg;
    const int r0 = static_cast<int>(gid - site * nrg) * RB;
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

    for (int dir = 0; dir < 81; ++dir) {
        if (dir == 40) continue;
        const int dx = dir % 3 - 1, dy = (dir / 3) % 3 - 1, dz = (dir / 9) % 3 - 1, dt = dir / 27 - 1;
        const int kh = (dx != 0) + (dy != 0) + (dz != 0) + (dt != 0);
        const R rho = static_cast<R>(DAG ? -c_rho[kh] : c_rho[kh]);
        const R q1 = rho * dx, q2 = rho * dy, q3 = rho * dz, q4 = rho * dt;
        const R lh = static_cast<R>(c_halflam[kh]);
        const int tt = c.t + dt;
        const int64_t nb = site_index(wrap(c.x + dx, g.nx), wrap(c.y + dy, g.ny), wrap(c.z + dz, g.nz),
                                      wrap(tt, g.nt), g);
        const R bsign = (g.apbc && (tt < 0 || tt >= g.nt)) ? R(-1) : R(1);

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
                // spin mixing: rows 0,1 get -lh ch + B ch_{2,3}; rows 2,3 get -lh ch + B^+ ch_{0,1}
                cx<R>* o = acc[k][a];
                // (q4 - i q3) ch2 + (-q2 - i q1) ch3
                o[0].re += -lh * ch[0].re + q4 * ch[2].re + q3 * ch[2].im - q2 * ch[3].re + q1 * ch[3].im;
                o[0].im += -lh * ch[0].im + q4 * ch[2].im - q3 * ch[2].re - q2 * ch[3].im - q1 * ch[3].re;
                // (q2 - i q1) ch2 + (q4 + i q3) ch3
                o[1].re += -lh * ch[1].re + q2 * ch[2].re + q1 * ch[2].im + q4 * ch[3].re - q3 * ch[3].im;
                o[1].im += -lh * ch[1].im + q2 * ch[2].im - q1 * ch[2].re + q4 * ch[3].im + q3 * ch[3].re;
                // (q4 + i q3) ch0 + (q2 + i q1) ch1
                o[2].re += -lh * ch[2].re + q4 * ch[0].re - q3 * ch[0].im + q2 * ch[1].re - q1 * ch[1].im;
                o[2].im += -lh * ch[2].im + q4 * ch[0].im + q3 * ch[0].re + q2 * ch[1].im + q1 * ch[1].re;
                // (-q2 + i q1) ch0 + (q4 - i q3) ch1
                o[3].re += -lh * ch[3].re - q2 * ch[0].re - q1 * ch[0].im + q4 * ch[1].re + q3 * ch[1].im;
                o[3].im += -lh * ch[3].im - q2 * ch[0].im + q1 * ch[0].re + q4 * ch[1].im - q3 * ch[1].re;
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
        hipLaunchKernelGGL((brillouin_kernel<NC, RB, true, P>), grid, dim3(block), 0, st, W, in, out, diag, a.g, a.nv);
    else
        hipLaunchKernelGGL((brillouin_kernel<NC, RB, false, P>), grid, dim3(block), 0, st, W, in, out, diag, a.g,
                           a.nv);
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
