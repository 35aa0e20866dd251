// Krylov solvers (Sec. 9) driving the stencil and BLAS-1 kernels.
//
// All N_v right-hand sides run in lock-step.  Per-RHS scalars (alpha, beta, norms) live in
// device memory; the host reads the N_v residual norms once per iteration (one stream
// synchronisation) to apply the paper's rules: the residual is recomputed explicitly
// every `recompute_every` iterations, when the updated residuals suggest convergence, and
// at the iteration limit; the solve ends when every recomputed residual meets the
// tolerance, when an updated and a recomputed norm differ by more than `drift`, or at the
// limit.  A converged RHS is frozen (zero step length).
//
// Mixed precision (outer FP64, inner FP32 or BF16): the paper wraps its single-precision
// solver in a double-precision updater (Sec. 9).  Two schemes:
//  * reliable updates (default): one CG in the inner precision whose residual is replaced
//    by the FP64 true residual b - A x whenever it has dropped by `delta` since the last
//    replacement; the solution is accumulated in FP64 and the search direction is kept;
//  * defect correction: restarted inner solves on the normalised FP64 residual.
// FP64 is kept for the true residual, the solution and every dot-product accumulation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace dirac {

namespace {

constexpr size_t kAlign = 256;

struct Carver {
    char* base;
    size_t cap;
    size_t used = 0;
    void* take(size_t bytes) {
        used = (used + kAlign - 1) / kAlign * kAlign;
        void* p = base ? base + used : nullptr;
        used += bytes;
        return p;
    }
};

struct OpCtx {
    dirac_op op;
    int nc, nv;
    Geom g;
    double mass;
    int64_t nrows;  // rows of nv complex per vector
    size_t ncomplex() const { return static_cast<size_t>(nrows) * nv; }
    // the Laplacians are hermitian positive definite: CG runs on D itself, not on D^+ D
    bool hermitian() const { return op_is_laplace(op); }
};

// The operator's links and (optional) clover field in one precision.
struct Field {
    const void* gauge;
    const void* clov;
};

size_t vec_bytes(const OpCtx& o, dirac_prec p) { return o.ncomplex() * complex_bytes(p); }

int apply_op(const OpCtx& o, dirac_prec p, const Field& f, const void* in, void* out, bool dag, hipStream_t st,
             const Epilogue& epi = Epilogue()) {
    return launch_stencil(o.op, p, o.nc, o.nv, o.g, o.mass, f.gauge, f.clov, in, out, dag, st, epi);
}

// out = A in with A = D^+ D via tmp (A = D for the hermitian Laplacians; tmp unused)
int apply_normal(const OpCtx& o, dirac_prec p, const Field& f, const void* in, void* out, void* tmp,
                 hipStream_t st) {
    if (o.hermitian()) return apply_op(o, p, f, in, out, false, st);
    int rc = apply_op(o, p, f, in, tmp, false, st);
    if (rc) return rc;
    return apply_op(o, p, f, tmp, out, true, st);
}

// Device scalar kernels (one thread per RHS).  alpha = rr / p^+ A p with p^+ A p = ||D p||^2
// (A = D^+ D), one double per RHS.
__global__ void k_cg_alpha(const double* __restrict__ pq, int pq_stride, const double* __restrict__ rr,
                           const double* __restrict__ mask, double* __restrict__ alpha, int nv) {
    const int i = threadIdx.x;
    if (i >= nv) return;
    const double d = pq[i * pq_stride];
    const bool ok = mask[i] != 0.0 && d > 0.0 && std::isfinite(d);
    alpha[2 * i] = ok ? rr[i] / d : 0.0;
    alpha[2 * i + 1] = 0.0;
}

// Line-search step of the reliable-update inner CG: alpha = <p, r> / p^+ A p = conj(<r, p>) / ||D p||^2,
// the exact minimiser along the stored direction p of the A-norm of the error.  With p stored in a
// lower precision than r, <r, p> drifts away from ||r||^2 (the deviation is carried forward by beta)
// and the textbook ||r||^2 / p^+ A p can then overshoot and make the recurrence diverge.
__global__ void k_cg_alpha_ls(const double* __restrict__ pq, int pq_stride, const double* __restrict__ rp,
                              const double* __restrict__ mask, double* __restrict__ alpha, int nv) {
    const int i = threadIdx.x;
    if (i >= nv) return;
    const double d = pq[i * pq_stride];
    const bool ok = mask[i] != 0.0 && d > 0.0 && std::isfinite(d);
    alpha[2 * i] = ok ? rp[2 * i] / d : 0.0;
    alpha[2 * i + 1] = ok ? -rp[2 * i + 1] / d : 0.0;
}

// beta = rr_new / rr (active RHS), then rr = rr_new
__global__ void k_cg_beta(const double* __restrict__ rr_new, double* __restrict__ rr, const double* __restrict__ mask,
                          double* __restrict__ beta, int nv) {
    const int i = threadIdx.x;
    if (i >= nv) return;
    const double old = rr[i];
    const bool ok = mask[i] != 0.0 && old > 0.0;
    beta[2 * i] = ok ? rr_new[i] / old : 0.0;
    beta[2 * i + 1] = 0.0;
    rr[i] = rr_new[i];
}

__global__ void k_fill(double* __restrict__ p, double v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Scalars and pinned host mirrors shared by one solve.
struct Scalars {
    int nv = 0;
    double* partial = nullptr;  // reduce_partial_doubles(nv)
    double* rr = nullptr;       // nv
    double* rr_new = nullptr;   // nv
    double* tmpn = nullptr;     // nv (norms of b, true residuals)
    double* pq = nullptr;       // 2nv
    double* alpha = nullptr;    // 2nv
    double* beta = nullptr;     // 2nv
    double* cplx = nullptr;     // 8nv general complex scratch (BiCGstab)
    double* mask = nullptr;     // nv (1 active, 0 frozen)
    double* rp = nullptr;       // 2nv: <r, p> (reliable-update line search)
    double* tiles = nullptr;    // ntiles * nv: per-tile partial sums of the stencil epilogues
    int64_t ntiles = 0;
    double* burst = nullptr;    // per-block partials of the one-pass x/p update with <r, p>
    size_t burst_doubles = 0;
    double* hbuf = nullptr;     // pinned host, 16 nv doubles
    void carve(Carver& c, int nv_, int64_t ntiles_, int64_t nrows) {
        nv = nv_;
        ntiles = ntiles_;
        tiles = static_cast<double*>(c.take(static_cast<size_t>(ntiles) * nv * sizeof(double)));
        burst_doubles = burst_partial_doubles(nrows, nv);
        burst = static_cast<double*>(c.take(burst_doubles * sizeof(double)));
        partial = static_cast<double*>(c.take(reduce_partial_doubles(nv) * sizeof(double)));
        rr = static_cast<double*>(c.take(nv * sizeof(double)));
        rr_new = static_cast<double*>(c.take(nv * sizeof(double)));
        tmpn = static_cast<double*>(c.take(nv * sizeof(double)));
        pq = static_cast<double*>(c.take(2 * nv * sizeof(double)));
        alpha = static_cast<double*>(c.take(2 * nv * sizeof(double)));
        beta = static_cast<double*>(c.take(2 * nv * sizeof(double)));
        cplx = static_cast<double*>(c.take(8 * nv * sizeof(double)));
        mask = static_cast<double*>(c.take(nv * sizeof(double)));
        rp = static_cast<double*>(c.take(2 * nv * sizeof(double)));
    }
};

// Pinned host staging buffer (grown on demand, kept for the process lifetime).
double* pinned(size_t ndoubles) {
    static thread_local double* buf = nullptr;
    static thread_local size_t cap = 0;
    if (ndoubles > cap) {
        if (buf) (void)hipHostFree(buf);
        buf = nullptr;
        cap = 0;
        if (hipHostMalloc(reinterpret_cast<void**>(&buf), ndoubles * sizeof(double), hipHostMallocDefault) !=
            hipSuccess)
            return nullptr;
        cap = ndoubles;
    }
    return buf;
}

int d2h(double* host, const double* dev, int n, hipStream_t st) {
    DIRAC_HIP(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, st));
    DIRAC_HIP(hipStreamSynchronize(st));
    return DIRAC_OK;
}
int h2d(double* dev, const double* host, int n, hipStream_t st) {
    DIRAC_HIP(hipMemcpyAsync(dev, host, n * sizeof(double), hipMemcpyHostToDevice, st));
    // the host buffer may be reused right away: make the copy complete
    DIRAC_HIP(hipStreamSynchronize(st));
    return DIRAC_OK;
}

struct Rules {
    double tol;
    int maxit;
    int recompute_every;
    double drift;
};

struct Result {
    int iters = 0;
    int recomputes = 0;
    int reason = 0;  // 0 converged, 1 stagnated, 2 maxit
    std::vector<double> relres;
    std::vector<double> alpha_hist, beta_hist;  // iteration-major, nv each
};

bool all_finite(const std::vector<double>& v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

// r = b - A x using q and t as temporaries (A = D^+ D in precision pp; x in px).
int residual_normal(const OpCtx& o, dirac_prec pp, const Field& f, dirac_prec pb, const void* b, dirac_prec px,
                    const void* x, dirac_prec pr, void* r, void* q, void* t, hipStream_t st) {
    const void* xin = x;
    if (px != pp) {
        int rc = blas_cast(px, x, pp, q, o.ncomplex(), st);
        if (rc) return rc;
        xin = q;
    }
    int rc = apply_normal(o, pp, f, xin, q, t, st);
    if (rc) return rc;
    return blas_sub(pb, b, pp, q, pr, r, o.ncomplex(), st);
}

// p^+ A p into s.pq after q = A p (and t = D p): ||t||^2 for A = D^+ D (one vector read instead of two),
// Re <p, q> for a hermitian A.  Returns the stride of the real values in s.pq.
int p_a_p(const OpCtx& o, dirac_prec pp, const void* p, const void* q, const void* t, double* partial, double* pq,
          int& stride, hipStream_t st) {
    if (o.hermitian()) {
        stride = 2;
        return blas_dot(pp, p, pp, q, o.nrows, o.nv, partial, pq, st);
    }
    stride = 1;
    return blas_norm2(pp, t, o.nrows, o.nv, partial, pq, st);
}

// The operator part of one CG step on A = D^+ D with the BLAS folded into the stencil epilogues:
// t = D p with the tiles' sums of |t|^2 (-> s.pq), the step length from `alpha_kernel`, then
// r -= alpha D^+ t with the tiles' sums of |r|^2 (-> s.rr_new); q = A p is never written.  kNoEpilogue
// (nothing launched) when the shape has no fused form: the caller then runs the separate kernels.
template <typename AlphaFn>
int fused_normal_step(const OpCtx& o, dirac_prec pp, const Field& f, const void* p, void* t, void* q, dirac_prec pr,
                      void* r, Scalars& s, AlphaFn&& alpha_kernel, hipStream_t st) {
    if (o.hermitian() || (pp == DIRAC_FP64) != (pr == DIRAC_FP64) || !s.tiles) return kNoEpilogue;
    Epilogue e1;
    e1.mode = 1;
    e1.partial = s.tiles;
    int rc = apply_op(o, pp, f, p, t, false, st, e1);
    if (rc) return rc;
    finalize_blocks(s.tiles, s.ntiles, o.nv, s.partial, s.pq, st);
    alpha_kernel();
    Epilogue e2;
    e2.mode = 2;
    e2.partial = s.tiles;
    e2.r = r;
    e2.alpha = s.alpha;
    if ((rc = apply_op(o, pp, f, t, q, true, st, e2))) return rc;
    finalize_blocks(s.tiles, s.ntiles, o.nv, s.partial, s.rr_new, st);
    return DIRAC_OK;
}

// ---------------------------------------------------------------------------
// CG core on A = D^+ D.  Vectors: x (px), r (pr), p, q, t (pp); b (pb); operator in pp.
// ---------------------------------------------------------------------------
struct CGVecs {
    const void* b;
    dirac_prec pb;
    void* x;
    dirac_prec px;
    void* r;
    dirac_prec pr;
    void *p, *q, *t;
    dirac_prec pp;
    Field f;
};

int cg_core(const OpCtx& o, const CGVecs& v, const Rules& ru, Scalars& s, hipStream_t st, Result& res,
            bool keep_history) {
    const int nv = o.nv;
    double* h = pinned(16 * nv);
    if (!h) return fail(DIRAC_EHIP, "hipHostMalloc of the solver staging buffer failed");
    int rc;
    // ||b||
    if ((rc = blas_norm2(v.pb, v.b, o.nrows, nv, s.partial, s.tmpn, st))) return rc;
    if ((rc = d2h(h, s.tmpn, nv, st))) return rc;
    std::vector<double> bn(nv), goal(nv);
    for (int i = 0; i < nv; ++i) {
        if (!std::isfinite(h[i])) return fail(DIRAC_ENONFINITE, "non-finite norm of the right-hand side");
        bn[i] = std::sqrt(h[i]);
        goal[i] = ru.tol * bn[i];
    }
    // r = b - A x ; rr
    if ((rc = residual_normal(o, v.pp, v.f, v.pb, v.b, v.px, v.x, v.pr, v.r, v.q, v.t, st))) return rc;
    if ((rc = blas_norm2(v.pr, v.r, o.nrows, nv, s.partial, s.rr, st))) return rc;
    if ((rc = d2h(h, s.rr, nv, st))) return rc;
    std::vector<double> rr(h, h + nv), active(nv);
    res.relres.assign(nv, 0.0);
    int nact = 0;
    for (int i = 0; i < nv; ++i) {
        if (!std::isfinite(rr[i])) return fail(DIRAC_ENONFINITE, "non-finite initial residual");
        active[i] = std::sqrt(rr[i]) > goal[i] ? 1.0 : 0.0;
        nact += active[i] != 0.0;
        res.relres[i] = bn[i] > 0 ? std::sqrt(rr[i]) / bn[i] : 0.0;
    }
    res.reason = 0;
    if (nact == 0) return DIRAC_OK;
    std::memcpy(h, active.data(), nv * sizeof(double));
    if ((rc = h2d(s.mask, h, nv, st))) return rc;
    // p = r
    if ((rc = blas_cast(v.pr, v.r, v.pp, v.p, o.ncomplex(), st))) return rc;

    int it = 0;
    while (true) {
        if (it >= ru.maxit) {
            res.reason = 2;
            break;
        }
        ++it;
        rc = fused_normal_step(o, v.pp, v.f, v.p, v.t, v.q, v.pr, v.r, s, [&]() {
            hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(256), 0, st, s.pq, 1, s.rr, s.mask, s.alpha, nv);
        }, st);
        if (rc == kNoEpilogue) {
            if ((rc = apply_normal(o, v.pp, v.f, v.p, v.q, v.t, st))) return rc;
            int pstride;
            if ((rc = p_a_p(o, v.pp, v.p, v.q, v.t, s.partial, s.pq, pstride, st))) return rc;
            hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(256), 0, st, s.pq, pstride, s.rr, s.mask, s.alpha, nv);
            if ((rc = fused_r_update(v.pr, v.r, v.pp, v.q, s.alpha, o.nrows, nv, s.partial, s.rr_new, st))) return rc;
        } else if (rc) {
            return rc;
        }
        if ((rc = d2h(h, s.rr_new, nv, st))) return rc;
        std::vector<double> rn(h, h + nv);
        if (!all_finite(rn)) return fail(DIRAC_ENONFINITE, "non-finite residual norm during CG");
        if (keep_history) {
            if ((rc = d2h(h, s.alpha, 2 * nv, st))) return rc;
            for (int i = 0; i < nv; ++i) res.alpha_hist.push_back(h[2 * i]);
        }
        bool suggest = true;
        for (int i = 0; i < nv; ++i)
            if (active[i] != 0.0 && std::sqrt(rn[i]) > goal[i]) suggest = false;
        const bool recompute = (it % ru.recompute_every == 0) || suggest || it == ru.maxit;
        if (!recompute) {
            hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(256), 0, st, s.rr_new, s.rr, s.mask, s.beta, nv);
            if (keep_history) {
                if ((rc = d2h(h, s.beta, 2 * nv, st))) return rc;
                for (int i = 0; i < nv; ++i) res.beta_hist.push_back(h[2 * i]);
            }
            if ((rc = fused_xp_update(v.px, v.x, v.pp, v.p, v.pr, v.r, s.alpha, s.beta, o.nrows, nv, st))) return rc;
            continue;
        }
        // x += alpha p, then the explicit residual
        if ((rc = blas_caxpy(v.pp, v.p, v.px, v.x, s.alpha, o.nrows, nv, st))) return rc;
        if ((rc = residual_normal(o, v.pp, v.f, v.pb, v.b, v.px, v.x, v.pr, v.r, v.q, v.t, st))) return rc;
        if ((rc = blas_norm2(v.pr, v.r, o.nrows, nv, s.partial, s.rr_new, st))) return rc;
        if ((rc = d2h(h, s.rr_new, nv, st))) return rc;
        std::vector<double> rt(h, h + nv);
        if (!all_finite(rt)) return fail(DIRAC_ENONFINITE, "non-finite recomputed residual");
        ++res.recomputes;
        bool stagnated = false;
        nact = 0;
        for (int i = 0; i < nv; ++i) {
            res.relres[i] = bn[i] > 0 ? std::sqrt(rt[i]) / bn[i] : 0.0;
            if (active[i] == 0.0) continue;
            const double gap = std::fabs(std::sqrt(rn[i]) - std::sqrt(rt[i])) / std::max(std::sqrt(rt[i]), 1e-300);
            if (std::sqrt(rt[i]) <= goal[i]) {
                active[i] = 0.0;
            } else {
                ++nact;
                if (gap > ru.drift) stagnated = true;
            }
        }
        std::memcpy(h, active.data(), nv * sizeof(double));
        if ((rc = h2d(s.mask, h, nv, st))) return rc;
        if (nact == 0) {
            res.reason = 0;
            break;
        }
        if (stagnated) {
            res.reason = 1;
            break;
        }
        if (it >= ru.maxit) {
            res.reason = 2;
            break;
        }
        hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(256), 0, st, s.rr_new, s.rr, s.mask, s.beta, nv);
        if (keep_history) {
            if ((rc = d2h(h, s.beta, 2 * nv, st))) return rc;
            for (int i = 0; i < nv; ++i) res.beta_hist.push_back(h[2 * i]);
        }
        // p = r + beta p
        if ((rc = blas_cxpay(v.pr, v.r, v.pp, v.p, s.beta, o.nrows, nv, st))) return rc;
    }
    res.iters = it;
    return DIRAC_OK;
}

// ---------------------------------------------------------------------------
// Reliable-update mixed CG: outer FP64 (x, b, r_hi, t_hi), inner r, xl (FP32) and p, q, t (pin).
// ---------------------------------------------------------------------------
struct RUVecs {
    const void* b;
    void* x;
    void *r_hi, *t_hi;
    void *r, *xl;
    void *p, *q, *t;
    dirac_prec pin;
    Field f_hi;
    Field f_lo;
};

int cg_reliable(const OpCtx& o, const RUVecs& v, const Rules& ru, double delta, Scalars& s, hipStream_t st,
                Result& res) {
    const int nv = o.nv;
    const dirac_prec F64 = DIRAC_FP64, F32 = DIRAC_FP32;
    double* h = pinned(16 * nv);
    if (!h) return fail(DIRAC_EHIP, "hipHostMalloc of the solver staging buffer failed");
    int rc;
    if ((rc = blas_norm2(F64, v.b, o.nrows, nv, s.partial, s.tmpn, st))) return rc;
    if ((rc = d2h(h, s.tmpn, nv, st))) return rc;
    std::vector<double> bn(nv), goal(nv);
    for (int i = 0; i < nv; ++i) {
        if (!std::isfinite(h[i])) return fail(DIRAC_ENONFINITE, "non-finite norm of the right-hand side");
        bn[i] = std::sqrt(h[i]);
        goal[i] = ru.tol * bn[i];
    }
    auto true_residual = [&](std::vector<double>& rt) -> int {
        int e;
        if ((e = apply_normal(o, F64, v.f_hi, v.x, v.r_hi, v.t_hi, st))) return e;
        if ((e = blas_bminus(F64, v.b, F64, v.r_hi, o.nrows, nv, st))) return e;
        if ((e = blas_norm2(F64, v.r_hi, o.nrows, nv, s.partial, s.tmpn, st))) return e;
        if ((e = d2h(h, s.tmpn, nv, st))) return e;
        rt.assign(h, h + nv);
        if (!all_finite(rt)) return fail(DIRAC_ENONFINITE, "non-finite FP64 residual");
        ++res.recomputes;
        return DIRAC_OK;
    };
    std::vector<double> rt, active(nv);
    if ((rc = true_residual(rt))) return rc;
    res.relres.assign(nv, 0.0);
    int nact = 0;
    for (int i = 0; i < nv; ++i) {
        res.relres[i] = bn[i] > 0 ? std::sqrt(rt[i]) / bn[i] : 0.0;
        active[i] = std::sqrt(rt[i]) > goal[i] ? 1.0 : 0.0;
        nact += active[i] != 0.0;
    }
    res.reason = 0;
    if (nact == 0) return DIRAC_OK;
    std::memcpy(h, active.data(), nv * sizeof(double));
    if ((rc = h2d(s.mask, h, nv, st))) return rc;
    const size_t n = o.ncomplex();
    // r = r_hi ; xl = 0 ; p = r ; rr = ||r||^2
    auto restart_inner = [&]() -> int {
        int e;
        if ((e = blas_cast(F64, v.r_hi, F32, v.r, n, st))) return e;
        DIRAC_HIP(hipMemsetAsync(v.xl, 0, n * complex_bytes(F32), st));
        if ((e = blas_norm2(F32, v.r, o.nrows, nv, s.partial, s.rr, st))) return e;
        return DIRAC_OK;
    };
    if ((rc = restart_inner())) return rc;
    if ((rc = blas_cast(F32, v.r, v.pin, v.p, n, st))) return rc;
    // <r, p> of the stored p: the numerator of the line-search step
    if ((rc = blas_dot(F32, v.r, v.pin, v.p, o.nrows, nv, s.partial, s.rp, st))) return rc;
    // rmax: largest inner residual norm since the last replacement (Sleijpen and van der Vorst)
    std::vector<double> rmax(nv), best(nv);
    for (int i = 0; i < nv; ++i) rmax[i] = best[i] = std::sqrt(rt[i]);
    std::vector<int> no_progress(nv, 0);

    int it = 0;
    while (true) {
        if (it >= ru.maxit) {
            res.reason = 2;
            break;
        }
        ++it;
        rc = fused_normal_step(o, v.pin, v.f_lo, v.p, v.t, v.q, F32, v.r, s, [&]() {
            hipLaunchKernelGGL(k_cg_alpha_ls, dim3(1), dim3(256), 0, st, s.pq, 1, s.rp, s.mask, s.alpha, nv);
        }, st);
        if (rc == kNoEpilogue) {
            if ((rc = apply_normal(o, v.pin, v.f_lo, v.p, v.q, v.t, st))) return rc;
            int pstride;
            if ((rc = p_a_p(o, v.pin, v.p, v.q, v.t, s.partial, s.pq, pstride, st))) return rc;
            hipLaunchKernelGGL(k_cg_alpha_ls, dim3(1), dim3(256), 0, st, s.pq, pstride, s.rp, s.mask, s.alpha, nv);
            if ((rc = fused_r_update(F32, v.r, v.pin, v.q, s.alpha, o.nrows, nv, s.partial, s.rr_new, st)))
                return rc;
        } else if (rc) {
            return rc;
        }
        if ((rc = d2h(h, s.rr_new, nv, st))) return rc;
        std::vector<double> rn(h, h + nv);
        if (!all_finite(rn)) return fail(DIRAC_ENONFINITE, "non-finite inner residual norm");
        bool update = it >= ru.maxit;
        bool suggest = true;
        for (int i = 0; i < nv; ++i) {
            if (active[i] == 0.0) continue;
            const double r_in = std::sqrt(rn[i]);
            rmax[i] = std::max(rmax[i], r_in);
            if (r_in < delta * rmax[i]) update = true;
            if (r_in > goal[i]) suggest = false;
        }
        update = update || suggest;
        hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(256), 0, st, s.rr_new, s.rr, s.mask, s.beta, nv);
        if ((rc = fused_xp_update_dot(F32, v.xl, v.pin, v.p, F32, v.r, s.alpha, s.beta, o.nrows, nv, s.partial, s.rp,
                                      st, s.burst, s.burst_doubles)))
            return rc;
        if (!update) continue;
        // x += xl in FP64, true residual, replace the inner residual (keep p)
        for (int i = 0; i < nv; ++i) {
            h[2 * i] = 1.0;
            h[2 * i + 1] = 0.0;
        }
        if ((rc = h2d(s.cplx, h, 2 * nv, st))) return rc;
        if ((rc = blas_caxpy(F32, v.xl, F64, v.x, s.cplx, o.nrows, nv, st))) return rc;
        if ((rc = true_residual(rt))) return rc;
        nact = 0;
        bool stuck = false;
        for (int i = 0; i < nv; ++i) {
            res.relres[i] = bn[i] > 0 ? std::sqrt(rt[i]) / bn[i] : 0.0;
            if (active[i] == 0.0) continue;
            const double rnow = std::sqrt(rt[i]);
            if (rnow <= goal[i]) {
                active[i] = 0.0;
                continue;
            }
            ++nact;
            if (rnow < 0.9 * best[i]) {
                best[i] = rnow;
                no_progress[i] = 0;
            } else if (++no_progress[i] >= 5) {
                stuck = true;
            }
            rmax[i] = rnow;
        }
        std::memcpy(h, active.data(), nv * sizeof(double));
        if ((rc = h2d(s.mask, h, nv, st))) return rc;
        if (nact == 0) {
            res.reason = 0;
            break;
        }
        if (stuck) {
            res.reason = 1;
            break;
        }
        if (it >= ru.maxit) {
            res.reason = 2;
            break;
        }
        if ((rc = restart_inner())) return rc;
        // p is kept; its line-search numerator is taken against the replaced residual
        if ((rc = blas_dot(F32, v.r, v.pin, v.p, o.nrows, nv, s.partial, s.rp, st))) return rc;
    }
    res.iters = it;
    return DIRAC_OK;
}

// ---------------------------------------------------------------------------
// BiCGstab core on D (van der Vorst 1992), all vectors in precision p, shadow r_hat = r_0.
// Per-RHS complex scalars are formed on the host.
// ---------------------------------------------------------------------------
struct BiVecs {
    const void* b;
    dirac_prec pb;
    void* x;
    void *r, *rhat, *p, *v, *s, *t;
    dirac_prec p_;
    Field f;
};

struct C {
    double re, im;
};
inline C cmulh(C a, C b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline C cdivh(C a, C b) {
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
inline double cabsh(C a) { return std::hypot(a.re, a.im); }

int bicgstab_core(const OpCtx& o, const BiVecs& v, const Rules& ru, Scalars& s, hipStream_t st, Result& res) {
    const int nv = o.nv;
    const dirac_prec P = v.p_;
    const size_t n = o.ncomplex();
    double* h = pinned(16 * nv);
    if (!h) return fail(DIRAC_EHIP, "hipHostMalloc of the solver staging buffer failed");
    int rc;
    if ((rc = blas_norm2(v.pb, v.b, o.nrows, nv, s.partial, s.tmpn, st))) return rc;
    if ((rc = d2h(h, s.tmpn, nv, st))) return rc;
    std::vector<double> bn(nv), goal(nv);
    for (int i = 0; i < nv; ++i) {
        if (!std::isfinite(h[i])) return fail(DIRAC_ENONFINITE, "non-finite norm of the right-hand side");
        bn[i] = std::sqrt(h[i]);
        goal[i] = ru.tol * bn[i];
    }
    auto residual = [&](std::vector<double>& rt) -> int {
        int e;
        if ((e = apply_op(o, P, v.f, v.x, v.t, false, st))) return e;
        if ((e = blas_sub(v.pb, v.b, P, v.t, P, v.r, n, st))) return e;
        if ((e = blas_norm2(P, v.r, o.nrows, nv, s.partial, s.tmpn, st))) return e;
        if ((e = d2h(h, s.tmpn, nv, st))) return e;
        rt.assign(h, h + nv);
        if (!all_finite(rt)) return fail(DIRAC_ENONFINITE, "non-finite recomputed residual");
        return DIRAC_OK;
    };
    auto dots = [&](const void* a, const void* b2, std::vector<C>& out) -> int {
        int e;
        if ((e = blas_dot(P, a, P, b2, o.nrows, nv, s.partial, s.pq, st))) return e;
        if ((e = d2h(h, s.pq, 2 * nv, st))) return e;
        out.resize(nv);
        for (int i = 0; i < nv; ++i) out[i] = {h[2 * i], h[2 * i + 1]};
        return DIRAC_OK;
    };
    auto norms = [&](const void* a, std::vector<double>& out) -> int {
        int e;
        if ((e = blas_norm2(P, a, o.nrows, nv, s.partial, s.tmpn, st))) return e;
        if ((e = d2h(h, s.tmpn, nv, st))) return e;
        out.assign(h, h + nv);
        return DIRAC_OK;
    };
    auto upload = [&](double* dev, const std::vector<C>& c) -> int {
        for (int i = 0; i < nv; ++i) {
            h[2 * i] = c[i].re;
            h[2 * i + 1] = c[i].im;
        }
        return h2d(dev, h, 2 * nv, st);
    };
    double* d_alpha = s.cplx;
    double* d_omega = s.cplx + 2 * nv;
    double* d_beta = s.cplx + 4 * nv;

    std::vector<double> rt;
    if ((rc = residual(rt))) return rc;
    res.relres.assign(nv, 0.0);
    std::vector<int> active(nv);
    int nact = 0;
    for (int i = 0; i < nv; ++i) {
        res.relres[i] = bn[i] > 0 ? std::sqrt(rt[i]) / bn[i] : 0.0;
        active[i] = std::sqrt(rt[i]) > goal[i];
        nact += active[i];
    }
    res.reason = 0;
    if (nact == 0) return DIRAC_OK;
    if ((rc = blas_cast(P, v.r, P, v.rhat, n, st))) return rc;
    DIRAC_HIP(hipMemsetAsync(v.p, 0, n * complex_bytes(P), st));
    DIRAC_HIP(hipMemsetAsync(v.v, 0, n * complex_bytes(P), st));
    std::vector<C> rho(nv, C{1, 0}), alpha(nv, C{1, 0}), omega(nv, C{1, 0}), beta(nv), tmpc, rv, ts;
    std::vector<double> rr(rt), rhn, tt, vn;
    int it = 0;
    while (true) {
        if (it >= ru.maxit) {
            res.reason = 2;
            break;
        }
        ++it;
        std::vector<C> rho_new;
        if ((rc = dots(v.rhat, v.r, rho_new))) return rc;
        if ((rc = norms(v.rhat, rhn))) return rc;
        // breakdown: restart that RHS with r_hat = r
        bool any_restart = false;
        std::vector<int> restart(nv, 0);
        for (int i = 0; i < nv; ++i) {
            if (!active[i]) continue;
            const double tiny = 1e-30 * std::sqrt(rhn[i] * rr[i]);
            if (cabsh(rho_new[i]) <= tiny || cabsh(omega[i]) == 0.0) {
                restart[i] = 1;
                any_restart = true;
            }
        }
        if (any_restart) {
            // r_hat_i = r_i, p_i = v_i = 0 for the restarted columns: x_i-scaled copies
            std::vector<C> keep(nv), zero(nv);
            for (int i = 0; i < nv; ++i) {
                keep[i] = restart[i] ? C{0, 0} : C{1, 0};
                zero[i] = restart[i] ? C{1, 0} : C{0, 0};
            }
            // rhat <- keep * rhat + restart * r ; p, v <- keep * (p, v)
            for (int i = 0; i < nv; ++i) h[i] = restart[i] ? 0.0 : 1.0;
            if ((rc = h2d(s.tmpn, h, nv, st))) return rc;
            if ((rc = blas_rscale(P, v.rhat, P, v.rhat, s.tmpn, o.nrows, nv, st))) return rc;
            if ((rc = blas_rscale(P, v.p, P, v.p, s.tmpn, o.nrows, nv, st))) return rc;
            if ((rc = blas_rscale(P, v.v, P, v.v, s.tmpn, o.nrows, nv, st))) return rc;
            if ((rc = upload(d_alpha, zero))) return rc;
            if ((rc = blas_caxpy(P, v.r, P, v.rhat, d_alpha, o.nrows, nv, st))) return rc;
            for (int i = 0; i < nv; ++i)
                if (restart[i]) {
                    rho_new[i] = {rr[i], 0.0};
                    rho[i] = alpha[i] = omega[i] = C{1, 0};
                }
        }
        for (int i = 0; i < nv; ++i)
            beta[i] = active[i] ? cmulh(cdivh(rho_new[i], rho[i]), cdivh(alpha[i], omega[i])) : C{0, 0};
        std::vector<C> om_act(nv);
        for (int i = 0; i < nv; ++i) om_act[i] = active[i] ? omega[i] : C{0, 0};
        if ((rc = upload(d_beta, beta))) return rc;
        if ((rc = upload(d_omega, om_act))) return rc;
        if ((rc = fused_bicg_p(P, v.p, v.r, v.v, d_beta, d_omega, o.nrows, nv, st))) return rc;
        if ((rc = apply_op(o, P, v.f, v.p, v.v, false, st))) return rc;
        if ((rc = dots(v.rhat, v.v, rv))) return rc;
        if ((rc = norms(v.v, vn))) return rc;
        for (int i = 0; i < nv; ++i) {
            const bool good = active[i] && cabsh(rv[i]) > 1e-30 * std::sqrt(rhn[i] * vn[i]);
            alpha[i] = good ? cdivh(rho_new[i], rv[i]) : C{0, 0};
        }
        if ((rc = upload(d_alpha, alpha))) return rc;
        if ((rc = fused_bicg_s(P, v.s, v.r, v.v, d_alpha, o.nrows, nv, st))) return rc;
        if ((rc = apply_op(o, P, v.f, v.s, v.t, false, st))) return rc;
        if ((rc = dots(v.t, v.s, ts))) return rc;
        if ((rc = norms(v.t, tt))) return rc;
        for (int i = 0; i < nv; ++i) {
            const bool ok = active[i] && tt[i] > 0.0 && (alpha[i].re != 0.0 || alpha[i].im != 0.0);
            omega[i] = ok ? C{ts[i].re / tt[i], ts[i].im / tt[i]} : C{0, 0};
            if (active[i]) rho[i] = rho_new[i];
        }
        if ((rc = upload(d_omega, omega))) return rc;
        if ((rc = fused_bicg_xr(P, v.x, v.p, v.s, v.t, v.r, d_alpha, d_omega, o.nrows, nv, s.partial, s.rr_new, st)))
            return rc;
        if ((rc = d2h(h, s.rr_new, nv, st))) return rc;
        std::vector<double> rn(h, h + nv);
        if (!all_finite(rn)) return fail(DIRAC_ENONFINITE, "non-finite residual norm during BiCGstab");
        bool suggest = true;
        for (int i = 0; i < nv; ++i)
            if (active[i] && std::sqrt(rn[i]) > goal[i]) suggest = false;
        rr = rn;
        if (!((it % ru.recompute_every == 0) || suggest || it == ru.maxit)) continue;
        if ((rc = residual(rt))) return rc;
        ++res.recomputes;
        bool stagnated = false;
        nact = 0;
        for (int i = 0; i < nv; ++i) {
            res.relres[i] = bn[i] > 0 ? std::sqrt(rt[i]) / bn[i] : 0.0;
            if (!active[i]) continue;
            const double gap = std::fabs(std::sqrt(rn[i]) - std::sqrt(rt[i])) / std::max(std::sqrt(rt[i]), 1e-300);
            if (std::sqrt(rt[i]) <= goal[i]) {
                active[i] = 0;
            } else {
                ++nact;
                if (gap > ru.drift) stagnated = true;
            }
        }
        rr = rt;
        if (nact == 0) {
            res.reason = 0;
            break;
        }
        if (stagnated) {
            res.reason = 1;
            break;
        }
        if (it >= ru.maxit) {
            res.reason = 2;
            break;
        }
        // frozen RHS: keep x, r unchanged from now on (zero alpha/omega through the active mask)
    }
    res.iters = it;
    return DIRAC_OK;
}

// Vector counts per scheme.
struct Layout {
    int n_hi = 0;   // FP64 vectors
    int n_f32 = 0;  // FP32 vectors
    int n_in = 0;   // inner-precision vectors
    int n_out = 0;  // outer-precision vectors (plain solves)
};

Layout layout_for(int solver, dirac_prec outer, dirac_prec inner, int scheme) {
    Layout l;
    const bool mixed = inner != outer;
    if (!mixed) {
        l.n_out = solver == 0 ? 4 : 6;
        return l;
    }
    if (solver == 0) {
        l.n_hi = 2;  // r_hi, t_hi
        if (scheme == 0) {
            l.n_f32 = 2;  // r, xl
            l.n_in = 3;   // p, q, t
        } else {
            l.n_f32 = 3;  // b_lo, x_lo, r_lo
            l.n_in = 3;   // p, q, t
        }
    } else {
        l.n_hi = 1;  // r_hi
        l.n_in = 8;  // b_lo, x_lo, r, rhat, p, v, s, t
    }
    return l;
}


// Defect correction: repeat { r = b - A x in FP64; stop if converged; x += |r| * e with e the
// inner-precision solution of A e = r/|r| } (the paper's "sp solver wrapped in a dp updater").
int defect_correction(const OpCtx& o, int solver, dirac_prec inner, const Field& f_hi, const Field& f_lo,
                      const void* b, void* x, double tol, int maxit, const Rules& ru, const dirac_solve_opts* opts,
                      Carver& c, Scalars& s, hipStream_t st, Result& res) {
    const int nv = o.nv;
    const size_t n = o.ncomplex();
    const int max_outer = (opts && opts->max_outer > 0) ? opts->max_outer : 100;
    const double inner_tol = (opts && opts->delta > 0) ? opts->delta : (inner == DIRAC_BF16 ? 5e-2 : 1e-5);
    void* r_hi = c.take(vec_bytes(o, DIRAC_FP64));
    void* t_hi = solver == 0 ? c.take(vec_bytes(o, DIRAC_FP64)) : nullptr;
    // inner right-hand side / solution precision: FP32 for CG (operator vectors in `inner`),
    // `inner` throughout for BiCGstab
    const dirac_prec pbl = solver == 0 ? DIRAC_FP32 : inner;
    void* b_lo = c.take(vec_bytes(o, pbl));
    void* x_lo = c.take(vec_bytes(o, pbl));
    void* r_lo = c.take(vec_bytes(o, pbl));
    void *p = c.take(vec_bytes(o, inner)), *q = c.take(vec_bytes(o, inner)), *t = c.take(vec_bytes(o, inner));
    void *rh = nullptr, *ss = nullptr;
    if (solver == 1) {
        rh = c.take(vec_bytes(o, inner));
        ss = c.take(vec_bytes(o, inner));
    }
    double* h = pinned(16 * nv);
    if (!h) return fail(DIRAC_EHIP, "hipHostMalloc of the solver staging buffer failed");
    int rc;
    if ((rc = blas_norm2(DIRAC_FP64, b, o.nrows, nv, s.partial, s.tmpn, st))) return rc;
    if ((rc = d2h(h, s.tmpn, nv, st))) return rc;
    std::vector<double> bn(nv), best(nv, HUGE_VAL);
    for (int i = 0; i < nv; ++i) {
        if (!std::isfinite(h[i])) return fail(DIRAC_ENONFINITE, "non-finite norm of the right-hand side");
        bn[i] = std::sqrt(h[i]);
    }
    Rules ir = ru;
    ir.tol = inner_tol;
    ir.recompute_every = 20;
    int total = 0, stall = 0;
    res.reason = 2;
    for (int outer_it = 0; outer_it <= max_outer; ++outer_it) {
        if (solver == 0) {
            if ((rc = apply_normal(o, DIRAC_FP64, f_hi, x, r_hi, t_hi, st))) return rc;
        } else {
            if ((rc = apply_op(o, DIRAC_FP64, f_hi, x, r_hi, false, st))) return rc;
        }
        if ((rc = blas_bminus(DIRAC_FP64, b, DIRAC_FP64, r_hi, o.nrows, nv, st))) return rc;
        if ((rc = blas_norm2(DIRAC_FP64, r_hi, o.nrows, nv, s.partial, s.tmpn, st))) return rc;
        if ((rc = d2h(h, s.tmpn, nv, st))) return rc;
        ++res.recomputes;
        std::vector<double> rn(h, h + nv);
        if (!all_finite(rn)) return fail(DIRAC_ENONFINITE, "non-finite FP64 residual");
        res.relres.assign(nv, 0.0);
        bool done = true, progress = false;
        for (int i = 0; i < nv; ++i) {
            const double nr = std::sqrt(rn[i]);
            res.relres[i] = bn[i] > 0 ? nr / bn[i] : 0.0;
            if (nr > tol * bn[i]) done = false;
            if (nr < 0.9 * best[i]) progress = true;
            best[i] = std::min(best[i], nr);
        }
        if (done) {
            res.reason = 0;
            break;
        }
        stall = progress ? 0 : stall + 1;
        if (stall >= 3) {
            res.reason = 1;
            break;
        }
        if (total >= maxit || outer_it == max_outer) {
            res.reason = 2;
            break;
        }
        // inner right-hand side r/|r| (zero for converged columns)
        for (int i = 0; i < nv; ++i) {
            const double nr = std::sqrt(rn[i]);
            h[i] = (nr > tol * bn[i] && nr > 0) ? 1.0 / nr : 0.0;
        }
        if ((rc = h2d(s.tmpn, h, nv, st))) return rc;
        if ((rc = blas_rscale(DIRAC_FP64, r_hi, pbl, b_lo, s.tmpn, o.nrows, nv, st))) return rc;
        DIRAC_HIP(hipMemsetAsync(x_lo, 0, n * complex_bytes(pbl), st));
        Result inner_res;
        Rules rr = ir;
        rr.maxit = std::max(1, maxit - total);
        if (solver == 0) {
            CGVecs v{b_lo, DIRAC_FP32, x_lo, DIRAC_FP32, r_lo, DIRAC_FP32, p, q, t, inner, f_lo};
            rc = cg_core(o, v, rr, s, st, inner_res, false);
        } else {
            BiVecs v{b_lo, inner, x_lo, r_lo, rh, p, q, ss, t, inner, f_lo};
            rc = bicgstab_core(o, v, rr, s, st, inner_res);
        }
        if (rc) return rc;
        total += inner_res.iters;
        // x += |r| e
        for (int i = 0; i < nv; ++i) {
            const double nr = std::sqrt(rn[i]);
            h[2 * i] = (nr > tol * bn[i]) ? nr : 0.0;
            h[2 * i + 1] = 0.0;
        }
        if ((rc = h2d(s.cplx, h, 2 * nv, st))) return rc;
        if ((rc = blas_caxpy(pbl, x_lo, DIRAC_FP64, x, s.cplx, o.nrows, nv, st))) return rc;
    }
    res.iters = total;
    return DIRAC_OK;
}

}  // namespace

size_t solver_workspace_bytes(dirac_op op, int solver, dirac_prec outer, dirac_prec inner, int nc, int nv,
                              const Geom& g, int scheme) {
    OpCtx o{op, nc, nv, g, 0.0, g.vol * nc * (op_four_spin(op) ? 4 : 1)};
    Layout l = layout_for(solver, outer, inner, scheme);
    Carver c{nullptr, 0};
    Scalars s;
    s.carve(c, nv, g.vol / g.nx, o.nrows);
    for (int i = 0; i < l.n_out; ++i) c.take(vec_bytes(o, outer));
    for (int i = 0; i < l.n_hi; ++i) c.take(vec_bytes(o, DIRAC_FP64));
    for (int i = 0; i < l.n_f32; ++i) c.take(vec_bytes(o, DIRAC_FP32));
    for (int i = 0; i < l.n_in; ++i) c.take(vec_bytes(o, inner));
    return c.used + kAlign;
}

int run_solver(int solver, dirac_op op, dirac_prec outer, dirac_prec inner, const void* gauge_hi,
               const void* gauge_lo, const void* clov_hi, const void* clov_lo, const void* b, void* x, double mass,
               int nc, int nv, const Geom& g, double tol, int maxit, void* workspace, size_t ws_bytes,
               dirac_solve_info* info, const dirac_solve_opts* opts, hipStream_t st) {
    const int scheme = opts ? opts->mixed_scheme : 0;
    if (ws_bytes < solver_workspace_bytes(op, solver, outer, inner, nc, nv, g, scheme))
        return fail(DIRAC_EWORKSPACE, "solver workspace smaller than dirac_solver_workspace_bytes()");
    OpCtx o{op, nc, nv, g, mass, g.vol * nc * (op_four_spin(op) ? 4 : 1)};
    const Field f_hi{gauge_hi, clov_hi};
    const Field f_lo{gauge_lo, clov_lo};
    // 256-byte align the carve base
    char* base = static_cast<char*>(workspace);
    const uintptr_t mis = reinterpret_cast<uintptr_t>(base) % kAlign;
    if (mis) base += kAlign - mis;
    Carver c{base, ws_bytes};
    Scalars s;
    s.carve(c, nv, g.vol / g.nx, o.nrows);
    const bool mixed = inner != outer;
    Rules ru;
    ru.tol = tol;
    ru.maxit = maxit;
    ru.recompute_every = (opts && opts->recompute_every > 0) ? opts->recompute_every : (outer == DIRAC_FP64 && !mixed ? 50 : 20);
    ru.drift = (opts && opts->drift > 0) ? opts->drift : 0.01;
    Result res;
    int rc = DIRAC_OK;
    const bool hist = info && info->alpha && info->beta && info->hist_cap > 0 && !mixed && solver == 0;
    if (!mixed) {
        if (solver == 0) {
            CGVecs v{b, outer, x, outer, c.take(vec_bytes(o, outer)), outer, c.take(vec_bytes(o, outer)),
                     c.take(vec_bytes(o, outer)), c.take(vec_bytes(o, outer)), outer, f_hi};
            v.pr = outer;
            rc = cg_core(o, v, ru, s, st, res, hist);
        } else {
            BiVecs v{b, outer, x, c.take(vec_bytes(o, outer)), c.take(vec_bytes(o, outer)), c.take(vec_bytes(o, outer)),
                     c.take(vec_bytes(o, outer)), c.take(vec_bytes(o, outer)), c.take(vec_bytes(o, outer)), outer,
                     f_hi};
            rc = bicgstab_core(o, v, ru, s, st, res);
        }
    } else if (solver == 0 && scheme == 0) {
        const double delta = (opts && opts->delta > 0) ? opts->delta : 0.1;
        RUVecs v;
        v.b = b;
        v.x = x;
        v.r_hi = c.take(vec_bytes(o, DIRAC_FP64));
        v.t_hi = c.take(vec_bytes(o, DIRAC_FP64));
        v.r = c.take(vec_bytes(o, DIRAC_FP32));
        v.xl = c.take(vec_bytes(o, DIRAC_FP32));
        v.p = c.take(vec_bytes(o, inner));
        v.q = c.take(vec_bytes(o, inner));
        v.t = c.take(vec_bytes(o, inner));
        v.pin = inner;
        v.f_hi = f_hi;
        v.f_lo = f_lo;
        rc = cg_reliable(o, v, ru, delta, s, st, res);
    } else {
        rc = defect_correction(o, solver, inner, f_hi, f_lo, b, x, tol, maxit, ru, opts, c, s, st, res);
    }
    if (rc) return rc;
    DIRAC_HIP(hipStreamSynchronize(st));
    if (info) {
        info->iters = res.iters;
        info->outer_iters = res.recomputes;
        info->reason = res.reason;
        if (info->true_relres)
            for (int i = 0; i < nv; ++i) info->true_relres[i] = i < static_cast<int>(res.relres.size()) ? res.relres[i] : 0.0;
        info->hist_len = 0;
        if (hist) {
            const int len = std::min<int>(info->hist_cap, static_cast<int>(res.beta_hist.size() / nv));
            for (int k = 0; k < len * nv; ++k) {
                info->alpha[k] = res.alpha_hist[k];
                info->beta[k] = res.beta_hist[k];
            }
            info->hist_len = len;
        }
    }
    return res.reason == 0 ? DIRAC_OK : DIRAC_NOT_CONVERGED;
}

}  // namespace dirac
