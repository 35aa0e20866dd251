// Stout smearing (Sec. 2; Morningstar and Peardon's analytic smearing) and the backward passes that
// carry a link gradient through it and through the Brillouin hypercube links W(V) (Tab. off-axis).
//
// One stout step, for every link at once from the old field:
//   C_mu(n)  = rho sum_{nu != mu} [U_nu(n) U_mu(n+nu) U_nu(n+mu)^+ + U_nu(n-nu)^+ U_mu(n-nu) U_nu(n-nu+mu)]
//   Omega    = C U^+,  Q = (i/2)(Omega^+ - Omega) - (i/(2N)) Tr(Omega^+ - Omega),  U' = exp(i Q) U.
// Gradients follow torch's convention for real losses: G = dL/dRe M + i dL/dIm M, so that
// dL = Re Tr(G^+ dM).  For a product the gradient of a factor is (left part)^+ G (right part)^+; for
// E = exp(X) it is L(X^+, G_E), the Frechet derivative of exp at X^+ in the direction G_E (the adjoint
// of L(X, .) for this inner product), read off the upper right block of exp([[X^+, G_E], [0, X^+]]).
// All arithmetic FP64 (complex128 links and gradients).  Gradients are accumulated with atomic adds, so
// the order of the additions (and the last bits of the result) can differ from run to run.
#include "common.h"
#include "kernels.h"

namespace dirac {

namespace {

template <int N>
struct CM {
    cx<double> e[N][N];
};

template <int N>
__device__ __forceinline__ CM<N> zero() {
    CM<N> r;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) r.e[i][j] = {0.0, 0.0};
    return r;
}

template <int N>
__device__ __forceinline__ CM<N> ident() {
    CM<N> r = zero<N>();
#pragma unroll
    for (int i = 0; i < N; ++i) r.e[i][i] = {1.0, 0.0};
    return r;
}

template <int N>
__device__ __forceinline__ CM<N> mul(const CM<N>& a, const CM<N>& b) {
    CM<N> r;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            cx<double> s{0.0, 0.0};
#pragma unroll
            for (int k = 0; k < N; ++k) cfma(s, a.e[i][k], b.e[k][j]);
            r.e[i][j] = s;
        }
    return r;
}

template <int N>
__device__ __forceinline__ CM<N> adj(const CM<N>& a) {
    CM<N> r;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) r.e[i][j] = cconj(a.e[j][i]);
    return r;
}

template <int N>
__device__ __forceinline__ void add_to(CM<N>& a, const CM<N>& b) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) a.e[i][j] = cadd(a.e[i][j], b.e[i][j]);
}

template <int N>
__device__ __forceinline__ CM<N> scaled(const CM<N>& a, cx<double> s) {
    CM<N> r;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) r.e[i][j] = cmul(s, a.e[i][j]);
    return r;
}

// exp(A) by scaling and squaring: A / 2^s with ||A / 2^s||_1 <= 1/4 (s from `norm_of`, so that a
// block whose off-diagonal part enters linearly can be scaled by its diagonal blocks alone), then an
// 18-term Taylor series, then s squarings.
template <int N>
__device__ CM<N> expm(const CM<N>& A, double norm_of) {
    int s = 0;
    double nrm = norm_of;
    while (nrm > 0.25 && s < 40) {
        nrm *= 0.5;
        ++s;
    }
    const double sc = ldexp(1.0, -s);
    const CM<N> X = scaled(A, cx<double>{sc, 0.0});
    CM<N> term = ident<N>(), sum = ident<N>();
    for (int k = 1; k <= 18; ++k) {
        term = scaled(mul(term, X), cx<double>{1.0 / k, 0.0});
        add_to(sum, term);
    }
    for (int i = 0; i < s; ++i) sum = mul(sum, sum);
    return sum;
}

// max column sum of |entries| of the leading n x n block
template <int N>
__device__ __forceinline__ double norm1(const CM<N>& a, int n) {
    double m = 0.0;
    for (int j = 0; j < n; ++j) {
        double c = 0.0;
        for (int i = 0; i < n; ++i) c += fabs(a.e[i][j].re) + fabs(a.e[i][j].im);
        m = c > m ? c : m;
    }
    return m;
}

template <int NC>
__device__ __forceinline__ CM<NC> load_link(const double2* __restrict__ U, int64_t site, int mu) {
    CM<NC> m;
    const double2* p = U + (site * 4 + mu) * NC * NC;
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            const double2 v = p[a * NC + b];
            m.e[a][b] = {v.x, v.y};
        }
    return m;
}

template <int NC>
__device__ __forceinline__ void atomic_add_link(double2* __restrict__ G, int64_t site, int mu, const CM<NC>& m) {
    double* p = reinterpret_cast<double*>(G + (site * 4 + mu) * NC * NC);
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            atomicAdd(p + 2 * (a * NC + b), m.e[a][b].re);
            atomicAdd(p + 2 * (a * NC + b) + 1, m.e[a][b].im);
        }
}

__device__ __forceinline__ int64_t shifted(const Coord& c, int mu, int s, const Geom& g) {
    int x[4] = {c.x, c.y, c.z, c.t};
    const int ext[4] = {g.nx, g.ny, g.nz, g.nt};
    x[mu] = wrap(x[mu] + s, ext[mu]);
    return site_index(x[0], x[1], x[2], x[3], g);
}

__device__ __forceinline__ int64_t shifted2(const Coord& c, int mu, int s, int nu, int t, const Geom& g) {
    int x[4] = {c.x, c.y, c.z, c.t};
    const int ext[4] = {g.nx, g.ny, g.nz, g.nt};
    x[mu] = wrap(x[mu] + s, ext[mu]);
    x[nu] = wrap(x[nu] + t, ext[nu]);
    return site_index(x[0], x[1], x[2], x[3], g);
}

// C_mu(n) / rho: the six staples
template <int NC>
__device__ CM<NC> staple_sum(const double2* __restrict__ U, int64_t site, const Coord& c, int mu, const Geom& g) {
    CM<NC> acc = zero<NC>();
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        const int64_t n_nu = shifted(c, nu, 1, g), n_mu = shifted(c, mu, 1, g);
        add_to(acc, mul(mul(load_link<NC>(U, site, nu), load_link<NC>(U, n_nu, mu)), adj(load_link<NC>(U, n_mu, nu))));
        const int64_t m_nu = shifted(c, nu, -1, g), m_nu_p_mu = shifted2(c, nu, -1, mu, 1, g);
        add_to(acc, mul(mul(adj(load_link<NC>(U, m_nu, nu)), load_link<NC>(U, m_nu, mu)), load_link<NC>(U, m_nu_p_mu, nu)));
    }
    return acc;
}

// X = i Q for the link (mu, n): Q = (i/2)(Omega^+ - Omega) minus its trace, Omega = C U^+
template <int NC>
__device__ __forceinline__ CM<NC> stout_x(const CM<NC>& C, const CM<NC>& Ul) {
    const CM<NC> om = mul(C, adj(Ul));
    CM<NC> a;  // Omega^+ - Omega (anti-hermitian)
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) a.e[i][j] = csub(cconj(om.e[j][i]), om.e[i][j]);
    cx<double> tr{0.0, 0.0};
#pragma unroll
    for (int i = 0; i < NC; ++i) tr = cadd(tr, a.e[i][i]);
#pragma unroll
    for (int i = 0; i < NC; ++i) a.e[i][i] = csub(a.e[i][i], cscale(1.0 / NC, tr));
    // X = i Q = i (i/2) a = -a/2
    return scaled(a, cx<double>{-0.5, 0.0});
}

template <int NC>
__global__ __launch_bounds__(128) void stout_kernel(const double2* __restrict__ U, double2* __restrict__ V, double rho,
                                                    Geom g) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= 4 * g.vol) return;
    const int64_t site = gid >> 2;
    const int mu = static_cast<int>(gid & 3);
    const Coord c = site_coord(site, g);
    const CM<NC> C = scaled(staple_sum<NC>(U, site, c, mu, g), cx<double>{rho, 0.0});
    const CM<NC> Ul = load_link<NC>(U, site, mu);
    const CM<NC> X = stout_x(C, Ul);
    const CM<NC> Vl = mul(expm(X, norm1(X, NC)), Ul);
    double2* out = V + (site * 4 + mu) * NC * NC;
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) out[a * NC + b] = make_double2(Vl.e[a][b].re, Vl.e[a][b].im);
}

// gU += the gradient with respect to U of L(U'(U)) given gV = dL/dU' (one stout step)
template <int NC>
__global__ __launch_bounds__(64) void stout_backward_kernel(const double2* __restrict__ U,
                                                            const double2* __restrict__ GV,
                                                            double2* __restrict__ GU, double rho, Geom g) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= 4 * g.vol) return;
    const int64_t site = gid >> 2;
    const int mu = static_cast<int>(gid & 3);
    const Coord c = site_coord(site, g);
    const CM<NC> C = scaled(staple_sum<NC>(U, site, c, mu, g), cx<double>{rho, 0.0});
    const CM<NC> Ul = load_link<NC>(U, site, mu);
    const CM<NC> X = stout_x(C, Ul);
    const double nx = norm1(X, NC);
    const CM<NC> E = expm(X, nx);
    const CM<NC> Gv = load_link<NC>(GV, site, mu);
    // V = E U: direct part E^+ G_V, and G_E = G_V U^+
    CM<NC> gu = mul(adj(E), Gv);
    const CM<NC> GE = mul(Gv, adj(Ul));
    // G_X = L(X^+, G_E) from the block exponential
    constexpr int N2 = 2 * NC;
    CM<N2> M = zero<N2>();
    const CM<NC> Xd = adj(X);
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            M.e[i][j] = Xd.e[i][j];
            M.e[NC + i][NC + j] = Xd.e[i][j];
            M.e[i][NC + j] = GE.e[i][j];
        }
    const CM<N2> EM = expm(M, nx);
    CM<NC> GX;
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) GX.e[i][j] = EM.e[i][NC + j];
    // X = i Q -> G_Q = -i G_X; Q = (i/2) A - (i/2N) Tr A -> G_A = (-i/2)(G_Q - Tr(G_Q)/N); A = Om^+ - Om ->
    // G_Om = G_A^+ - G_A; with G_Q = -i G_X: G_A = -(1/2)(G_X - Tr(G_X)/N)
    CM<NC> GA;
    cx<double> trx{0.0, 0.0};
#pragma unroll
    for (int i = 0; i < NC; ++i) trx = cadd(trx, GX.e[i][i]);
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            cx<double> v = GX.e[i][j];
            if (i == j) v = csub(v, cscale(1.0 / NC, trx));
            GA.e[i][j] = cscale(-0.5, v);
        }
    CM<NC> GOm;
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) GOm.e[i][j] = csub(cconj(GA.e[j][i]), GA.e[i][j]);
    // Omega = C U^+: G_C = G_Om U, and U gains G_Om^+ C
    add_to(gu, mul(adj(GOm), C));
    atomic_add_link<NC>(GU, site, mu, gu);
    const CM<NC> GP = scaled(mul(GOm, Ul), cx<double>{rho, 0.0});  // gradient of every staple product
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        {  // A B D = U_nu(n) U_mu(n+nu) U_nu(n+mu)^+
            const int64_t n_nu = shifted(c, nu, 1, g), n_mu = shifted(c, mu, 1, g);
            const CM<NC> A = load_link<NC>(U, site, nu), B = load_link<NC>(U, n_nu, mu),
                         D = adj(load_link<NC>(U, n_mu, nu));
            atomic_add_link<NC>(GU, site, nu, mul(GP, adj(mul(B, D))));
            atomic_add_link<NC>(GU, n_nu, mu, mul(mul(adj(A), GP), adj(D)));
            atomic_add_link<NC>(GU, n_mu, nu, adj(mul(adj(mul(A, B)), GP)));  // D = U^+: gradient daggered
        }
        {  // A B D = U_nu(n-nu)^+ U_mu(n-nu) U_nu(n-nu+mu)
            const int64_t m_nu = shifted(c, nu, -1, g), m_nu_p_mu = shifted2(c, nu, -1, mu, 1, g);
            const CM<NC> A = adj(load_link<NC>(U, m_nu, nu)), B = load_link<NC>(U, m_nu, mu),
                         D = load_link<NC>(U, m_nu_p_mu, nu);
            atomic_add_link<NC>(GU, m_nu, nu, adj(mul(GP, adj(mul(B, D)))));  // A = U^+
            atomic_add_link<NC>(GU, m_nu, mu, mul(mul(adj(A), GP), adj(D)));
            atomic_add_link<NC>(GU, m_nu_p_mu, nu, mul(adj(mul(A, B)), GP));
        }
    }
}

// gV += the gradient with respect to V of L(W(V)) given gW = dL/dW for the 40 stored directions:
// W_d(n) = (1/|d|!) sum over the orderings of the unit steps of the path products, a step -mu from x
// contributing V_mu(x-mu)^+.  One thread per (stored direction, site).
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

template <int NC>
__global__ __launch_bounds__(64) void links_backward_kernel(const double2* __restrict__ V, const double2* __restrict__ GW,
                                                            double2* __restrict__ GV, Geom g) {
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
    CM<NC> G;
    {
        const double2* p = GW + (site * 40 + dir) * NC * NC;
        for (int a = 0; a < NC; ++a)
            for (int b = 0; b < NC; ++b) G.e[a][b] = {p[a * NC + b].x, p[a * NC + b].y};
    }
    double fact = 1.0;
    for (int j = 2; j <= k; ++j) fact *= j;
    G = scaled(G, cx<double>{1.0 / fact, 0.0});
    int perm[4] = {0, 1, 2, 3};
    do {
        // the links of this path and the sites/directions of the V they come from
        CM<NC> L[4];
        int64_t lsite[4];
        int lmu[4];
        bool ladj[4];
        int x[4] = {c0.x, c0.y, c0.z, c0.t};
        for (int j = 0; j < k; ++j) {
            const int mu = smu[perm[j]];
            if (ssg[perm[j]] > 0) {
                lsite[j] = site_index(x[0], x[1], x[2], x[3], g);
                ladj[j] = false;
                x[mu] = wrap(x[mu] + 1, ext[mu]);
            } else {
                x[mu] = wrap(x[mu] - 1, ext[mu]);
                lsite[j] = site_index(x[0], x[1], x[2], x[3], g);
                ladj[j] = true;
            }
            lmu[j] = mu;
            const CM<NC> v = load_link<NC>(V, lsite[j], mu);
            L[j] = ladj[j] ? adj(v) : v;
        }
        // gradient of factor j: (L_0 .. L_{j-1})^+ G (L_{j+1} .. L_{k-1})^+
        CM<NC> pre = ident<NC>();
        for (int j = 0; j < k; ++j) {
            CM<NC> suf = ident<NC>();
            for (int l = j + 1; l < k; ++l) suf = mul(suf, L[l]);
            const CM<NC> gl = mul(mul(adj(pre), G), adj(suf));
            atomic_add_link<NC>(GV, lsite[j], lmu[j], ladj[j] ? adj(gl) : gl);
            pre = mul(pre, L[j]);
        }
    } while (next_perm(perm, k));
}

template <int NC>
int launch_nc(int which, const Geom& g, const void* a, const void* b, void* out, double rho, hipStream_t st) {
    auto A = static_cast<const double2*>(a);
    auto B = static_cast<const double2*>(b);
    auto O = static_cast<double2*>(out);
    if (which == 0) {
        const int block = 128;
        hipLaunchKernelGGL((stout_kernel<NC>), dim3(static_cast<unsigned>((4 * g.vol + block - 1) / block)),
                           dim3(block), 0, st, A, O, rho, g);
    } else if (which == 1) {
        const int block = 64;
        hipLaunchKernelGGL((stout_backward_kernel<NC>), dim3(static_cast<unsigned>((4 * g.vol + block - 1) / block)),
                           dim3(block), 0, st, A, B, O, rho, g);
    } else {
        const int block = 64;
        hipLaunchKernelGGL((links_backward_kernel<NC>), dim3(static_cast<unsigned>((40 * g.vol + block - 1) / block)),
                           dim3(block), 0, st, A, B, O, g);
    }
    return DIRAC_OK;
}

int dispatch(int which, int nc, const Geom& g, const void* a, const void* b, void* out, double rho, hipStream_t st) {
    switch (nc) {
        case 1: return launch_nc<1>(which, g, a, b, out, rho, st);
        case 2: return launch_nc<2>(which, g, a, b, out, rho, st);
        case 3: return launch_nc<3>(which, g, a, b, out, rho, st);
        case 4: return launch_nc<4>(which, g, a, b, out, rho, st);
    }
    return DIRAC_EUNSUPPORTED;
}

}  // namespace

int launch_stout(int nc, const Geom& g, const void* U, void* V, double rho, hipStream_t st) {
    return dispatch(0, nc, g, U, nullptr, V, rho, st);
}

int launch_stout_backward(int nc, const Geom& g, const void* U, const void* gV, void* gU, double rho, hipStream_t st) {
    return dispatch(1, nc, g, U, gV, gU, rho, st);
}

int launch_links_backward(int nc, const Geom& g, const void* V, const void* gW, void* gV, hipStream_t st) {
    return dispatch(2, nc, g, V, gW, gV, 0.0, st);
}

}  // namespace dirac
