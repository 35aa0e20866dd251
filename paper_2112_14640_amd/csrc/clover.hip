// Clover field (Sec. 4, Eq. def_clov): the per-site chiral blocks of
//   C(n) = -(c_SW/2) sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}(n)
// from the links, in the packed form of clover.h.  F_{mu nu}(n) is the clover-leaf field strength:
// Q = the four plaquettes of the (mu, nu) plane that start and end at n, each run first along mu then
// along nu, and F = (Q - Q^+)/(8i) with its trace removed (traceless hermitian).  Computed in FP64,
// one thread per site; stored in the arithmetic type of the apply.
#include "clover.h"
#include "common.h"
#include "kernels.h"

namespace dirac {

namespace {

template <int NC>
struct Mat {
    cx<double> e[NC][NC];
};

template <int NC>
__device__ __forceinline__ Mat<NC> mul(const Mat<NC>& a, const Mat<NC>& b) {
    Mat<NC> r;
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            cx<double> s{0.0, 0.0};
#pragma unroll
            for (int k = 0; k < NC; ++k) cfma(s, a.e[i][k], b.e[k][j]);
            r.e[i][j] = s;
        }
    return r;
}

// U_mu at the site with coordinates c (periodic), as stored or as its adjoint
template <int NC, typename GI>
__device__ __forceinline__ Mat<NC> link(const GI* __restrict__ U, const int (&c)[4], int mu, bool adj, const Geom& g) {
    const int64_t s = site_index(c[0], c[1], c[2], c[3], g);
    const GI* p = U + (s * 4 + mu) * NC * NC;
    Mat<NC> m;
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            const cx<double> v = io<double, GI>::ld(p + a * NC + b);
            if (adj)
                m.e[b][a] = cconj(v);
            else
                m.e[a][b] = v;
        }
    return m;
}

__device__ __forceinline__ void step(int (&c)[4], int mu, int s, const int (&ext)[4]) { c[mu] = wrap(c[mu] + s, ext[mu]); }

// Q_{mu nu}(n): the four leaves, each a closed loop from n
template <int NC, typename GI>
__device__ Mat<NC> leaves(const GI* __restrict__ U, const int (&n)[4], int mu, int nu, const Geom& g) {
    const int ext[4] = {g.nx, g.ny, g.nz, g.nt};
    Mat<NC> q;
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) q.e[a][b] = {0.0, 0.0};
    auto add = [&](const Mat<NC>& m) {
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int b = 0; b < NC; ++b) q.e[a][b] = cadd(q.e[a][b], m.e[a][b]);
    };
    // n -> n+mu -> n+mu+nu -> n+nu -> n
    {
        int cm[4] = {n[0], n[1], n[2], n[3]};
        step(cm, mu, 1, ext);
        int cn[4] = {n[0], n[1], n[2], n[3]};
        step(cn, nu, 1, ext);
        Mat<NC> m = mul(link<NC>(U, n, mu, false, g), link<NC>(U, cm, nu, false, g));
        m = mul(m, link<NC>(U, cn, mu, true, g));
        add(mul(m, link<NC>(U, n, nu, true, g)));
    }
    // n -> n+nu -> n+nu-mu -> n-mu -> n
    {
        int cnm[4] = {n[0], n[1], n[2], n[3]};
        step(cnm, nu, 1, ext);
        step(cnm, mu, -1, ext);
        int cm[4] = {n[0], n[1], n[2], n[3]};
        step(cm, mu, -1, ext);
        Mat<NC> m = mul(link<NC>(U, n, nu, false, g), link<NC>(U, cnm, mu, true, g));
        m = mul(m, link<NC>(U, cm, nu, true, g));
        add(mul(m, link<NC>(U, cm, mu, false, g)));
    }
    // n -> n-mu -> n-mu-nu -> n-nu -> n
    {
        int cm[4] = {n[0], n[1], n[2], n[3]};
        step(cm, mu, -1, ext);
        int cmn[4] = {cm[0], cm[1], cm[2], cm[3]};
        step(cmn, nu, -1, ext);
        int cn[4] = {n[0], n[1], n[2], n[3]};
        step(cn, nu, -1, ext);
        Mat<NC> m = mul(link<NC>(U, cm, mu, true, g), link<NC>(U, cmn, nu, true, g));
        m = mul(m, link<NC>(U, cmn, mu, false, g));
        add(mul(m, link<NC>(U, cn, nu, false, g)));
    }
    // n -> n-nu -> n-nu+mu -> n+mu -> n
    {
        int cn[4] = {n[0], n[1], n[2], n[3]};
        step(cn, nu, -1, ext);
        int cnp[4] = {cn[0], cn[1], cn[2], cn[3]};
        step(cnp, mu, 1, ext);
        Mat<NC> m = mul(link<NC>(U, cn, nu, true, g), link<NC>(U, cn, mu, false, g));
        m = mul(m, link<NC>(U, cnp, nu, false, g));
        add(mul(m, link<NC>(U, n, mu, true, g)));
    }
    return q;
}

// F = (Q - Q^+)/(8i) minus trace/NC
template <int NC>
__device__ __forceinline__ Mat<NC> field_from(const Mat<NC>& q) {
    Mat<NC> f;
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            const cx<double> d = csub(q.e[a][b], cconj(q.e[b][a]));
            f.e[a][b] = {0.125 * d.im, -0.125 * d.re};  // d / (8 i)
        }
    double tr = 0.0;
#pragma unroll
    for (int a = 0; a < NC; ++a) tr += f.e[a][a].re;
#pragma unroll
    for (int a = 0; a < NC; ++a) f.e[a][a].re -= tr / NC;
    return f;
}

template <int NC, typename GI, typename CO>
__global__ __launch_bounds__(128) void clover_field_kernel(const GI* __restrict__ U, CO* __restrict__ out, double csw,
                                                           Geom g) {
    const int64_t site = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (site >= g.vol) return;
    const Coord co = site_coord(site, g);
    const int n[4] = {co.x, co.y, co.z, co.t};
    // planes (mu, nu), 0-based: 0 (0,1) 1 (0,2) 2 (0,3) 3 (1,2) 4 (1,3) 5 (2,3)
    const Mat<NC> f12 = field_from(leaves<NC>(U, n, 0, 1, g));
    const Mat<NC> f13 = field_from(leaves<NC>(U, n, 0, 2, g));
    const Mat<NC> f14 = field_from(leaves<NC>(U, n, 0, 3, g));
    const Mat<NC> f23 = field_from(leaves<NC>(U, n, 1, 2, g));
    const Mat<NC> f24 = field_from(leaves<NC>(U, n, 1, 3, g));
    const Mat<NC> f34 = field_from(leaves<NC>(U, n, 2, 3, g));
    constexpr int N = 2 * NC;
    const double s = -0.5 * csw;
    CO* o = out + site * clover_reals<NC>();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double sg = h == 0 ? 1.0 : -1.0;
        // block_h = s [[C, A - i B], [A + i B, -C]] with A = sg F14 - F23, B = F13 + sg F24, C = sg F34 - F12
        auto entry = [&](int i, int j) {
            const int si = i / NC, sj = j / NC, a = i % NC, b = j % NC;
            const cx<double> A{sg * f14.e[a][b].re - f23.e[a][b].re, sg * f14.e[a][b].im - f23.e[a][b].im};
            const cx<double> B{f13.e[a][b].re + sg * f24.e[a][b].re, f13.e[a][b].im + sg * f24.e[a][b].im};
            const cx<double> C{sg * f34.e[a][b].re - f12.e[a][b].re, sg * f34.e[a][b].im - f12.e[a][b].im};
            cx<double> v;
            if (si == 0 && sj == 0)
                v = C;
            else if (si == 1 && sj == 1)
                v = {-C.re, -C.im};
            else if (si == 0)
                v = {A.re + B.im, A.im - B.re};  // A - i B
            else
                v = {A.re - B.im, A.im + B.re};  // A + i B
            return cx<double>{s * v.re, s * v.im};
        };
        CO* blk = o + h * N * N;
#pragma unroll
        for (int i = 0; i < N; ++i) blk[i] = static_cast<CO>(entry(i, i).re);
        int e = N;
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = i + 1; j < N; ++j) {
                const cx<double> v = entry(i, j);
                blk[e] = static_cast<CO>(v.re);
                blk[e + 1] = static_cast<CO>(v.im);
                e += 2;
            }
    }
}

template <int NC>
void launch_nc(dirac_prec prec, const Geom& g, const void* U, void* C, double csw, hipStream_t st) {
    const int block = 128;
    const dim3 grid(static_cast<unsigned>((g.vol + block - 1) / block));
    if (prec == DIRAC_FP64)
        hipLaunchKernelGGL((clover_field_kernel<NC, double2, double>), grid, dim3(block), 0, st,
                           static_cast<const double2*>(U), static_cast<double*>(C), csw, g);
    else
        hipLaunchKernelGGL((clover_field_kernel<NC, float2, float>), grid, dim3(block), 0, st,
                           static_cast<const float2*>(U), static_cast<float*>(C), csw, g);
}

}  // namespace

size_t clover_field_reals(int nc) {
    return static_cast<size_t>(2) * (2 * nc) * (2 * nc);
}

int launch_clover_field(dirac_prec prec, int nc, const Geom& g, const void* U, void* C, double csw, hipStream_t st) {
    switch (nc) {
        case 1: launch_nc<1>(prec, g, U, C, csw, st); break;
        case 2: launch_nc<2>(prec, g, U, C, csw, st); break;
        case 3: launch_nc<3>(prec, g, U, C, csw, st); break;
        case 4: launch_nc<4>(prec, g, U, C, csw, st); break;
        default: return DIRAC_EUNSUPPORTED;
    }
    return DIRAC_OK;
}

}  // namespace dirac
