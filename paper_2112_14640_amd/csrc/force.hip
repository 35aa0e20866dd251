// Link gradients of Dirac bilinears and their su(Nc) projection (FP64).
//
// Gradient convention: for real L, g = dL/dRe U + i dL/dIm U.  For L = Re sum_rhs psi^+ D chi:
//   Wilson (from Eq. app_wils; U_mu(n) appears in the hops n -> n+mu and n+mu -> n):
//     g_mu(n) = -1/2 b sum_{s,rhs} [((1 - g_mu) psi(n))_s chi_s(n+mu)^+ + chi_s(n) ((1 + g_mu) psi(n+mu))_s^+]
//   Staggered (Eq. def_stag):
//     g_mu(n) = 1/2 eta_mu(n) b sum_rhs [psi(n) chi(n+mu)^+ - chi(n) psi(n+mu)^+]
//   Brillouin (Eq. app_bril), for each stored link W_d(n) (d one of the 40 stored directions), which
//   enters the hop n -> n+d as W_d(n) and the hop n+d -> n as W_{-d}(n+d) = W_d(n)^+:
//     g_d(n) = b sum_{s,rhs} [psi(n) (S_d chi(n+d))^+ + (psi(n+d) (S_{-d} chi(n))^+)^+]  (colour outer
//     products), with S_d = rho_|d| sum_mu d_mu g_mu - lambda_|d|/2 the spin factor of displacement d.
// b is the fermion boundary sign of the hop n -> n+mu (n -> n+d).  One thread per link; the kernel
// accumulates coeff * g into the output (each link written by exactly one thread).
#include "common.h"
#include "kernels.h"

namespace dirac {

namespace {

// g_mu p in the chiral basis (App. A), all four rows.
__device__ __forceinline__ void gamma_rows(int mu, const cx<double> p[4], cx<double> gp[4]) {
    switch (mu) {
        case 0:  // g1 = [[0,0,0,-i],[0,0,-i,0],[0,i,0,0],[i,0,0,0]]
            gp[0] = cscale(-1.0, cmuli(p[3]));
            gp[1] = cscale(-1.0, cmuli(p[2]));
            gp[2] = cmuli(p[1]);
            gp[3] = cmuli(p[0]);
            break;
        case 1:  // g2 = [[0,0,0,-1],[0,0,1,0],[0,1,0,0],[-1,0,0,0]]
            gp[0] = cscale(-1.0, p[3]);
            gp[1] = p[2];
            gp[2] = p[1];
            gp[3] = cscale(-1.0, p[0]);
            break;
        case 2:  // g3 = [[0,0,-i,0],[0,0,0,i],[i,0,0,0],[0,-i,0,0]]
            gp[0] = cscale(-1.0, cmuli(p[2]));
            gp[1] = cmuli(p[3]);
            gp[2] = cmuli(p[0]);
            gp[3] = cscale(-1.0, cmuli(p[1]));
            break;
        default:  // g4 = [[0,0,1,0],[0,0,0,1],[1,0,0,0],[0,1,0,0]]
            gp[0] = p[2];
            gp[1] = p[3];
            gp[2] = p[0];
            gp[3] = p[1];
            break;
    }
}

// (1 + SIG g_mu) p for the chiral basis, all four rows (SIG = +1 or -1).
__device__ __forceinline__ void spin_proj_full(int mu, double sig, const cx<double> p[4], cx<double> o[4]) {
    cx<double> gp[4];
    gamma_rows(mu, p, gp);
    for (int s = 0; s < 4; ++s) o[s] = cadd(p[s], cscale(sig, gp[s]));
}

// o = (rho sum_mu d_mu g_mu - lh) p, the Brillouin spin factor at displacement d (lh = lambda_|d|/2)
__device__ __forceinline__ void brillouin_spin(const int (&d)[4], double rho, double lh, const cx<double> p[4],
                                               cx<double> o[4]) {
    for (int s = 0; s < 4; ++s) o[s] = cscale(-lh, p[s]);
    for (int mu = 0; mu < 4; ++mu) {
        if (d[mu] == 0) continue;
        cx<double> gp[4];
        gamma_rows(mu, p, gp);
        for (int s = 0; s < 4; ++s) o[s] = cadd(o[s], cscale(rho * d[mu], gp[s]));
    }
}

// One thread per (stored direction, site): g_d(n) for W_d(n), see the file header.
template <int NC>
__global__ __launch_bounds__(128) void brillouin_force_kernel(const double2* __restrict__ psi,
                                                               const double2* __restrict__ chi,
                                                               double2* __restrict__ gout, double coeff, Geom g,
                                                               int nv) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= 40 * g.vol) return;
    const int dir = static_cast<int>(gid / g.vol);
    const int64_t site = gid - static_cast<int64_t>(dir) * g.vol;
    const int d[4] = {dir % 3 - 1, (dir / 3) % 3 - 1, (dir / 9) % 3 - 1, dir / 27 - 1};
    const int md[4] = {-d[0], -d[1], -d[2], -d[3]};
    const int k = (d[0] != 0) + (d[1] != 0) + (d[2] != 0) + (d[3] != 0);
    const double rho_k[5] = {0.0, 64.0 / 432.0, 16.0 / 432.0, 4.0 / 432.0, 1.0 / 432.0};
    const double lh_k[5] = {-120.0 / 64.0, 4.0 / 64.0, 2.0 / 64.0, 1.0 / 64.0, 0.5 / 64.0};
    const Coord c = site_coord(site, g);
    const int nbx = wrap(c.x + d[0], g.nx), nby = wrap(c.y + d[1], g.ny), nbz = wrap(c.z + d[2], g.nz);
    const int tt = c.t + d[3];
    const int nbt = wrap(tt, g.nt);
    const int64_t nb = site_index(nbx, nby, nbz, nbt, g);
    const double b = (g.apbc && (tt < 0 || tt >= g.nt)) ? -1.0 : 1.0;  // the same for the hop back
    const int64_t vs = static_cast<int64_t>(NC) * 4 * nv;

    cx<double> acc[NC][NC], bck[NC][NC];
    for (int a = 0; a < NC; ++a)
        for (int bb = 0; bb < NC; ++bb) acc[a][bb] = bck[a][bb] = {0.0, 0.0};
    for (int r = 0; r < nv; ++r) {
        cx<double> sc_nb[NC][4], sc_n[NC][4];
        for (int a = 0; a < NC; ++a) {
            cx<double> p_nb[4], p_n[4];
            for (int s = 0; s < 4; ++s) {
                p_nb[s] = io<double, double2>::ld(chi + nb * vs + (a * 4 + s) * nv + r);
                p_n[s] = io<double, double2>::ld(chi + site * vs + (a * 4 + s) * nv + r);
            }
            brillouin_spin(d, rho_k[k], lh_k[k], p_nb, sc_nb[a]);
            brillouin_spin(md, rho_k[k], lh_k[k], p_n, sc_n[a]);
        }
        for (int a = 0; a < NC; ++a)
            for (int s = 0; s < 4; ++s) {
                const cx<double> pn = io<double, double2>::ld(psi + site * vs + (a * 4 + s) * nv + r);
                const cx<double> pb = io<double, double2>::ld(psi + nb * vs + (a * 4 + s) * nv + r);
                for (int bb = 0; bb < NC; ++bb) {
                    cfma_conj(acc[a][bb], sc_nb[bb][s], pn);  // psi(n)_a conj(S_d chi(n+d))_b
                    cfma_conj(bck[a][bb], sc_n[bb][s], pb);   // psi(n+d)_a conj(S_-d chi(n))_b
                }
            }
    }
    const double f = b * coeff;
    double2* o = gout + (site * 40 + dir) * NC * NC;
    for (int a = 0; a < NC; ++a)
        for (int bb = 0; bb < NC; ++bb) {
            const cx<double> v = cadd(acc[a][bb], cconj(bck[bb][a]));
            double2 w = o[a * NC + bb];
            w.x += f * v.re;
            w.y += f * v.im;
            o[a * NC + bb] = w;
        }
}

template <int NC>
__global__ __launch_bounds__(256) void wilson_force_kernel(const double2* __restrict__ psi, const double2* __restrict__ chi,
                                                            double2* __restrict__ gout, double coeff, Geom g, int nv) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= 4 * g.vol) return;
    const int64_t site = gid >> 2;
    const int mu = static_cast<int>(gid & 3);
    const Coord c = site_coord(site, g);
    const int coord[4] = {c.x, c.y, c.z, c.t};
    const int ext[4] = {g.nx, g.ny, g.nz, g.nt};
    const int64_t stride[4] = {1, g.nx, static_cast<int64_t>(g.nx) * g.ny, static_cast<int64_t>(g.nx) * g.ny * g.nz};
    const int64_t fwd = site + (coord[mu] == ext[mu] - 1 ? (1 - ext[mu]) * stride[mu] : stride[mu]);
    double b = 1.0;
    if (mu == 3 && g.apbc && c.t == g.nt - 1) b = -1.0;
    const int64_t vs = static_cast<int64_t>(NC) * 4 * nv;

    cx<double> acc[NC][NC];
    for (int a = 0; a < NC; ++a)
        for (int bb = 0; bb < NC; ++bb) acc[a][bb] = {0.0, 0.0};
    for (int r = 0; r < nv; ++r) {
        cx<double> pm[NC][4], pp[NC][4], cn[NC][4], cf[NC][4];
        for (int a = 0; a < NC; ++a) {
            cx<double> p0[4], p1[4];
            for (int s = 0; s < 4; ++s) {
                p0[s] = io<double, double2>::ld(psi + site * vs + (a * 4 + s) * nv + r);
                p1[s] = io<double, double2>::ld(psi + fwd * vs + (a * 4 + s) * nv + r);
                cn[a][s] = io<double, double2>::ld(chi + site * vs + (a * 4 + s) * nv + r);
                cf[a][s] = io<double, double2>::ld(chi + fwd * vs + (a * 4 + s) * nv + r);
            }
            spin_proj_full(mu, -1.0, p0, pm[a]);
            spin_proj_full(mu, +1.0, p1, pp[a]);
        }
        for (int a = 0; a < NC; ++a)
            for (int bb = 0; bb < NC; ++bb)
                for (int s = 0; s < 4; ++s) {
                    // ((1-g)psi(n))_a conj(chi(n+mu))_b + chi(n)_a conj((1+g)psi(n+mu))_b
                    cfma_conj(acc[a][bb], cf[bb][s], pm[a][s]);
                    cfma_conj(acc[a][bb], pp[bb][s], cn[a][s]);
                }
    }
    const double f = -0.5 * b * coeff;
    double2* o = gout + (site * 4 + mu) * NC * NC;
    for (int a = 0; a < NC; ++a)
        for (int bb = 0; bb < NC; ++bb) {
            double2 v = o[a * NC + bb];
            v.x += f * acc[a][bb].re;
            v.y += f * acc[a][bb].im;
            o[a * NC + bb] = v;
        }
}

template <int NC>
__global__ __launch_bounds__(256) void staggered_force_kernel(const double2* __restrict__ psi,
                                                               const double2* __restrict__ chi,
                                                               double2* __restrict__ gout, double coeff, Geom g,
                                                               int nv) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= 4 * g.vol) return;
    const int64_t site = gid >> 2;
    const int mu = static_cast<int>(gid & 3);
    const Coord c = site_coord(site, g);
    const int coord[4] = {c.x, c.y, c.z, c.t};
    const int ext[4] = {g.nx, g.ny, g.nz, g.nt};
    const int64_t stride[4] = {1, g.nx, static_cast<int64_t>(g.nx) * g.ny, static_cast<int64_t>(g.nx) * g.ny * g.nz};
    const int64_t fwd = site + (coord[mu] == ext[mu] - 1 ? (1 - ext[mu]) * stride[mu] : stride[mu]);
    double b = 1.0;
    if (mu == 3 && g.apbc && c.t == g.nt - 1) b = -1.0;
    const int par = mu == 0 ? 0 : (mu == 1 ? (c.x & 1) : (mu == 2 ? ((c.x + c.y) & 1) : ((c.x + c.y + c.z) & 1)));
    const double eta = par ? -1.0 : 1.0;
    const int64_t vs = static_cast<int64_t>(NC) * nv;

    cx<double> acc[NC][NC];
    for (int a = 0; a < NC; ++a)
        for (int bb = 0; bb < NC; ++bb) acc[a][bb] = {0.0, 0.0};
    for (int r = 0; r < nv; ++r) {
        cx<double> p0[NC], p1[NC], c0[NC], c1[NC];
        for (int a = 0; a < NC; ++a) {
            p0[a] = io<double, double2>::ld(psi + site * vs + a * nv + r);
            p1[a] = io<double, double2>::ld(psi + fwd * vs + a * nv + r);
            c0[a] = io<double, double2>::ld(chi + site * vs + a * nv + r);
            c1[a] = io<double, double2>::ld(chi + fwd * vs + a * nv + r);
        }
        for (int a = 0; a < NC; ++a)
            for (int bb = 0; bb < NC; ++bb) {
                cfma_conj(acc[a][bb], c1[bb], p0[a]);  // psi(n)_a conj(chi(n+mu))_b
                cx<double> t{0.0, 0.0};
                cfma_conj(t, p1[bb], c0[a]);  // chi(n)_a conj(psi(n+mu))_b
                acc[a][bb] = csub(acc[a][bb], t);
            }
    }
    const double f = 0.5 * eta * b * coeff;
    double2* o = gout + (site * 4 + mu) * NC * NC;
    for (int a = 0; a < NC; ++a)
        for (int bb = 0; bb < NC; ++bb) {
            double2 v = o[a * NC + bb];
            v.x += f * acc[a][bb].re;
            v.y += f * acc[a][bb].im;
            o[a * NC + bb] = v;
        }
}

// F = (i/2)(U g^+ - g U^+) - tr/Nc
template <int NC>
__global__ __launch_bounds__(256) void project_kernel(const double2* __restrict__ U, const double2* g,
                                                       double2* F, int64_t nlinks) {
    const int64_t l = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (l >= nlinks) return;
    cx<double> u[NC][NC], gg[NC][NC], m[NC][NC];
    for (int a = 0; a < NC; ++a)
        for (int b = 0; b < NC; ++b) {
            u[a][b] = io<double, double2>::ld(U + l * NC * NC + a * NC + b);
            gg[a][b] = io<double, double2>::ld(g + l * NC * NC + a * NC + b);
        }
    // M = U g^+ ; F = (i/2)(M - M^+)
    for (int a = 0; a < NC; ++a)
        for (int b = 0; b < NC; ++b) {
            cx<double> s{0.0, 0.0};
            for (int e = 0; e < NC; ++e) cfma_conj(s, gg[b][e], u[a][e]);  // u[a][e] conj(g[b][e])
            m[a][b] = s;
        }
    cx<double> tr{0.0, 0.0};
    cx<double> f[NC][NC];
    for (int a = 0; a < NC; ++a)
        for (int b = 0; b < NC; ++b) {
            cx<double> d = csub(m[a][b], cconj(m[b][a]));
            f[a][b] = cscale(0.5, cmuli(d));
        }
    for (int a = 0; a < NC; ++a) tr = cadd(tr, f[a][a]);
    tr = cscale(1.0 / NC, tr);
    for (int a = 0; a < NC; ++a) f[a][a] = csub(f[a][a], tr);
    for (int a = 0; a < NC; ++a)
        for (int b = 0; b < NC; ++b) io<double, double2>::st(F + l * NC * NC + a * NC + b, f[a][b]);
}

template <int NC>
void launch_force_nc(dirac_op op, int nv, const Geom& g, const void* psi, const void* chi, void* gout, double coeff,
                     hipStream_t st) {
    const int block = 256;
    const dim3 grid(static_cast<unsigned>((4 * g.vol + block - 1) / block));
    if (op == DIRAC_WILSON)
        hipLaunchKernelGGL((wilson_force_kernel<NC>), grid, dim3(block), 0, st, static_cast<const double2*>(psi),
                           static_cast<const double2*>(chi), static_cast<double2*>(gout), coeff, g, nv);
    else
        hipLaunchKernelGGL((staggered_force_kernel<NC>), grid, dim3(block), 0, st, static_cast<const double2*>(psi),
                           static_cast<const double2*>(chi), static_cast<double2*>(gout), coeff, g, nv);
}

}  // namespace

template <int NC>
void launch_bforce_nc(int nv, const Geom& g, const void* psi, const void* chi, void* gout, double coeff,
                      hipStream_t st) {
    const int block = 128;
    const dim3 grid(static_cast<unsigned>((40 * g.vol + block - 1) / block));
    hipLaunchKernelGGL((brillouin_force_kernel<NC>), grid, dim3(block), 0, st, static_cast<const double2*>(psi),
                       static_cast<const double2*>(chi), static_cast<double2*>(gout), coeff, g, nv);
}

int launch_force(dirac_op op, int nc, int nv, const Geom& g, const void* /*U*/, const void* psi, const void* chi,
                 void* gout, double coeff, hipStream_t st) {
    if (op == DIRAC_BRILLOUIN) {
        switch (nc) {
            case 1: launch_bforce_nc<1>(nv, g, psi, chi, gout, coeff, st); break;
            case 2: launch_bforce_nc<2>(nv, g, psi, chi, gout, coeff, st); break;
            case 3: launch_bforce_nc<3>(nv, g, psi, chi, gout, coeff, st); break;
            case 4: launch_bforce_nc<4>(nv, g, psi, chi, gout, coeff, st); break;
            default: return DIRAC_EUNSUPPORTED;
        }
        return DIRAC_OK;
    }
    switch (nc) {
        case 1: launch_force_nc<1>(op, nv, g, psi, chi, gout, coeff, st); break;
        case 2: launch_force_nc<2>(op, nv, g, psi, chi, gout, coeff, st); break;
        case 3: launch_force_nc<3>(op, nv, g, psi, chi, gout, coeff, st); break;
        case 4: launch_force_nc<4>(op, nv, g, psi, chi, gout, coeff, st); break;
        default: return DIRAC_EUNSUPPORTED;
    }
    return DIRAC_OK;
}

int launch_project_su(int nc, int64_t nlinks, const void* U, const void* g, void* F, hipStream_t st) {
    const int block = 256;
    const dim3 grid(static_cast<unsigned>((nlinks + block - 1) / block));
    auto u = static_cast<const double2*>(U);
    auto gg = static_cast<const double2*>(g);
    auto f = static_cast<double2*>(F);
    switch (nc) {
        case 1: hipLaunchKernelGGL((project_kernel<1>), grid, dim3(block), 0, st, u, gg, f, nlinks); break;
        case 2: hipLaunchKernelGGL((project_kernel<2>), grid, dim3(block), 0, st, u, gg, f, nlinks); break;
        case 3: hipLaunchKernelGGL((project_kernel<3>), grid, dim3(block), 0, st, u, gg, f, nlinks); break;
        case 4: hipLaunchKernelGGL((project_kernel<4>), grid, dim3(block), 0, st, u, gg, f, nlinks); break;
        default: return DIRAC_EUNSUPPORTED;
    }
    return DIRAC_OK;
}

}  // namespace dirac
