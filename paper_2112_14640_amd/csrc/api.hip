// C ABI of libdirac: argument validation, dispatch to the kernel launchers and error strings.
// Validation runs before any launch; no entry point throws or aborts.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>

#include "common.h"
#include "kernels.h"

namespace dirac {

namespace {
thread_local std::string g_last_error;

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

bool aligned(const void* p, size_t a) { return reinterpret_cast<uintptr_t>(p) % a == 0; }

// Launch-shape overrides, [op][prec]; 0 = automatic.
constexpr int kOps = 5;
int g_rb_override[kOps][3] = {};
int g_variant_override[kOps][3] = {};

int check_common(dirac_op op, dirac_prec prec, int nc, int nv, const dirac_dims* dims, Geom& g) {
    if (op < DIRAC_WILSON || op > DIRAC_BRILLOUIN_LAPLACE) return fail(DIRAC_EINVAL, "unknown operator");
    if (prec < DIRAC_FP64 || prec > DIRAC_BF16) return fail(DIRAC_EINVAL, "unknown precision");
    if (!dims) return fail(DIRAC_EINVAL, "dims is NULL");
    for (int mu = 0; mu < 4; ++mu) {
        if (dims->n[mu] < 2) return fail(DIRAC_EINVAL, "lattice extents must be >= 2");
        if (op == DIRAC_STAGGERED && (dims->n[mu] & 1)) return fail(DIRAC_EINVAL, "staggered extents must be even");
    }
    if (nv < 1 || nv > 256) return fail(DIRAC_EINVAL, "nv must be in 1..256");
    if (nc < 1 || nc > 4) return fail(DIRAC_EUNSUPPORTED, "nc must be in 1..4");
    g.nx = dims->n[0];
    g.ny = dims->n[1];
    g.nz = dims->n[2];
    g.nt = dims->n[3];
    g.vol = static_cast<int64_t>(g.nx) * g.ny * g.nz * g.nt;
    if (g.vol >= (int64_t(1) << 31)) return fail(DIRAC_EINVAL, "lattice volume must be below 2^31 sites");
    g.apbc = dims->antiperiodic_t ? 1 : 0;
    return DIRAC_OK;
}

int64_t rows_of(dirac_op op, int nc, const Geom& g) { return g.vol * nc * (op_four_spin(op) ? 4 : 1); }

size_t gauge_bytes(dirac_op op, dirac_prec prec, int nc, const Geom& g) {
    const int dirs = op_uses_w(op) ? 40 : 4;
    return static_cast<size_t>(g.vol) * dirs * nc * nc * gauge_complex_bytes(prec);
}

size_t clover_bytes(dirac_prec prec, int nc, const Geom& g) {
    return static_cast<size_t>(g.vol) * clover_field_reals(nc) * (prec == DIRAC_FP64 ? 8 : 4);
}

int stencil(dirac_op op, dirac_prec prec, const void* gauge, const void* clover, const void* u, void* v, double mass,
            int nc, int nv, const dirac_dims* dims, void* stream, bool dag) {
    Geom g;
    int rc = check_common(op, prec, nc, nv, dims, g);
    if (rc) return rc;
    if (!gauge || !u || !v) return fail(DIRAC_EINVAL, "NULL gauge or vector pointer");
    const size_t vb = static_cast<size_t>(rows_of(op, nc, g)) * nv * complex_bytes(prec);
    if (overlap(u, vb, v, vb)) return fail(DIRAC_EINVAL, "input and output vectors overlap");
    if (overlap(gauge, gauge_bytes(op, prec, nc, g), v, vb)) return fail(DIRAC_EINVAL, "gauge and output overlap");
    if (!aligned(u, complex_bytes(prec)) || !aligned(v, complex_bytes(prec)) ||
        !aligned(gauge, gauge_complex_bytes(prec)))
        return fail(DIRAC_EINVAL, "misaligned pointer");
    if (clover) {
        if (!op_takes_clover(op)) return fail(DIRAC_EINVAL, "the clover term belongs to Wilson and Brillouin");
        if (!aligned(clover, prec == DIRAC_FP64 ? 8 : 4)) return fail(DIRAC_EINVAL, "misaligned clover field");
        if (overlap(clover, clover_bytes(prec, nc, g), v, vb)) return fail(DIRAC_EINVAL, "clover and output overlap");
    }
    if (!std::isfinite(mass)) return fail(DIRAC_EINVAL, "mass is not finite");
    rc = launch_stencil(op, prec, nc, nv, g, mass, gauge, clover, u, v, dag, as_stream(stream));
    if (rc) return fail(rc, "stencil launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

int check_hip(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return DIRAC_EHIP;
}

// Default launch shapes, chosen by timing the shapes at 16^3 x 32 and 32^3 x 64, Nc = 3, Nv = 12 on
// MI355X:
//   Wilson: row tiles (one x-row per work-group staged in LDS), 1 RHS per thread (2 where a row of
//           single-RHS threads would exceed 512 threads); with Nv = 12 each direction's links are
//           staged in LDS beside the row and the RHS stride is a compile-time constant.
//   staggered: row tiles, 2 RHS per thread (4 where 2 would exceed 512 threads per row); FP32 and
//              BF16 stage each direction's links in LDS, FP64 loads them per thread.
//   Wilson Laplacian: the staggered row kernel on 4 Nv columns, 4 per thread.
//   Brillouin (and its Laplacian): 1 RHS per thread; FP32 and BF16 row tiles (27 row copies per
//              x-row, link windows in LDS), FP64 direct loads (the row tile spills registers in FP64).
// Row tiles fall back to direct loads for shapes they cannot take; an rb that does not divide the
// columns falls back to 1.
int choose_rb(dirac_op op, dirac_prec prec, int nc, int nv, const Geom& g) {
    (void)nc;
    const int cols = op == DIRAC_WILSON_LAPLACE ? 4 * nv : nv;
    const int o = g_rb_override[op][prec];
    if (o > 0) return cols % o == 0 ? o : 1;
    switch (op) {
        case DIRAC_WILSON:
            return (static_cast<int64_t>(g.nx) * nv > 512 && nv % 2 == 0) ? 2 : 1;
        case DIRAC_STAGGERED: {
            if (cols % 2 != 0) return 1;
            return (static_cast<int64_t>(g.nx) * cols / 2 > 512 && cols % 4 == 0) ? 4 : 2;
        }
        case DIRAC_WILSON_LAPLACE:
            return 4;
        default:
            return 1;
    }
}

// 1 = direct loads, 4 = row tiles (see dirac_set_launch_shape)
int choose_variant(dirac_op op, dirac_prec prec) {
    const int o = g_variant_override[op][prec];
    if (o > 0) return o;
    return 4;
}

int launch_stencil(dirac_op op, dirac_prec prec, int nc, int nv, const Geom& g, double mass, const void* gauge,
                   const void* clover, const void* in, void* out, bool dag, hipStream_t st, const Epilogue& epi) {
    StencilArgs a{prec, nc, nv, choose_rb(op, prec, nc, nv, g), choose_variant(op, prec), dag, mass, g, gauge, in, out};
    a.clover = op_takes_clover(op) ? clover : nullptr;
    a.laplace = op_is_laplace(op);
    if (epi.mode != 0) {
        // the solver epilogues exist on the Wilson and staggered row kernels only
        if (op != DIRAC_WILSON && op != DIRAC_STAGGERED) return kNoEpilogue;
        a.epi = epi;
    }
    if (a.laplace) a.dagger = false;  // hermitian
    switch (op) {
        case DIRAC_WILSON: return launch_wilson(a, st);
        case DIRAC_BRILLOUIN:
        case DIRAC_BRILLOUIN_LAPLACE: return launch_brillouin(a, st);
        case DIRAC_STAGGERED:
        case DIRAC_WILSON_LAPLACE: return launch_staggered(a, st);
    }
    return DIRAC_EINVAL;
}

size_t solver_workspace_bytes(dirac_op op, int solver, dirac_prec outer, dirac_prec inner, int nc, int nv,
                              const Geom& g, int scheme);
int run_solver(int solver, dirac_op op, dirac_prec outer, dirac_prec inner, const void* gauge_hi,
               const void* gauge_lo, const void* clov_hi, const void* clov_lo, const void* b, void* x, double mass,
               int nc, int nv, const Geom& g, double tol, int maxit, void* workspace, size_t ws_bytes,
               dirac_solve_info* info, const dirac_solve_opts* opts, hipStream_t st);

}  // namespace dirac

using namespace dirac;

extern "C" {

int dirac_apply(dirac_op op, dirac_prec prec, const void* gauge, const void* u, void* v, double mass, int nc, int nv,
                const dirac_dims* dims, void* stream) {
    return stencil(op, prec, gauge, nullptr, u, v, mass, nc, nv, dims, stream, false);
}

int dirac_apply_dagger(dirac_op op, dirac_prec prec, const void* gauge, const void* u, void* v, double mass, int nc,
                       int nv, const dirac_dims* dims, void* stream) {
    return stencil(op, prec, gauge, nullptr, u, v, mass, nc, nv, dims, stream, true);
}

int dirac_apply_clover(dirac_op op, dirac_prec prec, const void* gauge, const void* clover, const void* u, void* v,
                       double mass, int nc, int nv, const dirac_dims* dims, void* stream) {
    if (!clover) return fail(DIRAC_EINVAL, "NULL clover field");
    return stencil(op, prec, gauge, clover, u, v, mass, nc, nv, dims, stream, false);
}

int dirac_apply_clover_dagger(dirac_op op, dirac_prec prec, const void* gauge, const void* clover, const void* u,
                              void* v, double mass, int nc, int nv, const dirac_dims* dims, void* stream) {
    if (!clover) return fail(DIRAC_EINVAL, "NULL clover field");
    return stencil(op, prec, gauge, clover, u, v, mass, nc, nv, dims, stream, true);
}

size_t dirac_clover_field_bytes(dirac_prec prec, int nc, const dirac_dims* dims) {
    Geom g;
    if (check_common(DIRAC_WILSON, prec, nc, 1, dims, g)) return 0;
    return clover_bytes(prec, nc, g);
}

int dirac_clover_field(dirac_prec prec, const void* U, double csw, void* clover, int nc, const dirac_dims* dims,
                       void* stream) {
    Geom g;
    int rc = check_common(DIRAC_WILSON, prec, nc, 1, dims, g);
    if (rc) return rc;
    if (!U || !clover) return fail(DIRAC_EINVAL, "NULL pointer");
    if (!std::isfinite(csw)) return fail(DIRAC_EINVAL, "c_SW is not finite");
    if (!aligned(U, gauge_complex_bytes(prec)) || !aligned(clover, prec == DIRAC_FP64 ? 8 : 4))
        return fail(DIRAC_EINVAL, "misaligned pointer");
    if (overlap(U, gauge_bytes(DIRAC_WILSON, prec, nc, g), clover, clover_bytes(prec, nc, g)))
        return fail(DIRAC_EINVAL, "U and the clover field overlap");
    rc = launch_clover_field(prec, nc, g, U, clover, csw, as_stream(stream));
    if (rc) return fail(rc, "clover launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

int dirac_apply_normal(dirac_op op, dirac_prec prec, const void* gauge, const void* u, void* v, void* tmp,
                       double mass, int nc, int nv, const dirac_dims* dims, void* stream) {
    Geom g;
    int rc = check_common(op, prec, nc, nv, dims, g);
    if (rc) return rc;
    if (!tmp) return fail(DIRAC_EINVAL, "NULL scratch vector");
    const size_t vb = static_cast<size_t>(rows_of(op, nc, g)) * nv * complex_bytes(prec);
    if (u && (overlap(u, vb, tmp, vb) || (v && overlap(v, vb, tmp, vb))))
        return fail(DIRAC_EINVAL, "scratch vector overlaps input or output");
    if (op_is_laplace(op)) return stencil(op, prec, gauge, nullptr, u, v, mass, nc, nv, dims, stream, false);
    rc = stencil(op, prec, gauge, nullptr, u, tmp, mass, nc, nv, dims, stream, false);
    if (rc) return rc;
    return stencil(op, prec, gauge, nullptr, tmp, v, mass, nc, nv, dims, stream, true);
}

int dirac_brillouin_links(dirac_prec prec, const void* U, void* W, int nc, const dirac_dims* dims, void* stream) {
    Geom g;
    int rc = check_common(DIRAC_BRILLOUIN, prec, nc, 1, dims, g);
    if (rc) return rc;
    if (!U || !W) return fail(DIRAC_EINVAL, "NULL link pointer");
    if (overlap(U, gauge_bytes(DIRAC_WILSON, prec, nc, g), W, gauge_bytes(DIRAC_BRILLOUIN, prec, nc, g)))
        return fail(DIRAC_EINVAL, "U and W overlap");
    if (!aligned(U, gauge_complex_bytes(prec)) || !aligned(W, gauge_complex_bytes(prec)))
        return fail(DIRAC_EINVAL, "misaligned pointer");
    rc = launch_brillouin_links(prec, nc, g, U, W, as_stream(stream));
    if (rc) return fail(rc, "link launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

int dirac_force(dirac_op op, const void* U, const void* psi, const void* chi, void* gout, double coeff, int nc, int nv,
                const dirac_dims* dims, void* stream) {
    Geom g;
    int rc = check_common(op, DIRAC_FP64, nc, nv, dims, g);
    if (rc) return rc;
    if (op != DIRAC_WILSON && op != DIRAC_STAGGERED && op != DIRAC_BRILLOUIN)
        return fail(DIRAC_EUNSUPPORTED, "force is implemented for the Wilson, Brillouin and staggered operators");
    if (!psi || !chi || !gout) return fail(DIRAC_EINVAL, "NULL pointer");
    const size_t vb = static_cast<size_t>(rows_of(op, nc, g)) * nv * 16;
    const size_t gb = gauge_bytes(op, DIRAC_FP64, nc, g);
    if (overlap(psi, vb, gout, gb) || overlap(chi, vb, gout, gb)) return fail(DIRAC_EINVAL, "output overlaps inputs");
    rc = launch_force(op, nc, nv, g, U, psi, chi, gout, coeff, as_stream(stream));
    if (rc) return fail(rc, "force launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

// The smearing and link-gradient calls share these checks: FP64 links, extents, no overlap of the
// output with the inputs.
static int link_call(const void* in1, bool two_inputs, const void* in2, void* out, int nc, const dirac_dims* dims,
                     Geom& g) {
    int rc = check_common(DIRAC_WILSON, DIRAC_FP64, nc, 1, dims, g);
    if (rc) return rc;
    if (!in1 || !out || (two_inputs && !in2)) return fail(DIRAC_EINVAL, "NULL pointer");
    if (!aligned(in1, 16) || !aligned(out, 16) || (in2 && !aligned(in2, 16)))
        return fail(DIRAC_EINVAL, "misaligned pointer");
    return DIRAC_OK;
}

int dirac_stout_smear(const void* U, void* V, double rho, int nc, const dirac_dims* dims, void* stream) {
    Geom g;
    int rc = link_call(U, false, nullptr, V, nc, dims, g);
    if (rc) return rc;
    if (!std::isfinite(rho)) return fail(DIRAC_EINVAL, "rho is not finite");
    const size_t b = gauge_bytes(DIRAC_WILSON, DIRAC_FP64, nc, g);
    if (overlap(U, b, V, b)) return fail(DIRAC_EINVAL, "U and V overlap");
    rc = launch_stout(nc, g, U, V, rho, as_stream(stream));
    if (rc) return fail(rc, "stout launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

int dirac_stout_backward(const void* U, const void* gV, void* gU, double rho, int nc, const dirac_dims* dims,
                         void* stream) {
    Geom g;
    int rc = link_call(U, true, gV, gU, nc, dims, g);
    if (rc) return rc;
    if (!std::isfinite(rho)) return fail(DIRAC_EINVAL, "rho is not finite");
    const size_t b = gauge_bytes(DIRAC_WILSON, DIRAC_FP64, nc, g);
    if (overlap(U, b, gU, b) || overlap(gV, b, gU, b)) return fail(DIRAC_EINVAL, "gU overlaps U or gV");
    rc = launch_stout_backward(nc, g, U, gV, gU, rho, as_stream(stream));
    if (rc) return fail(rc, "stout backward launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

int dirac_brillouin_links_backward(const void* V, const void* gW, void* gV, int nc, const dirac_dims* dims,
                                   void* stream) {
    Geom g;
    int rc = link_call(V, true, gW, gV, nc, dims, g);
    if (rc) return rc;
    const size_t bv = gauge_bytes(DIRAC_WILSON, DIRAC_FP64, nc, g);
    const size_t bw = gauge_bytes(DIRAC_BRILLOUIN, DIRAC_FP64, nc, g);
    if (overlap(V, bv, gV, bv) || overlap(gW, bw, gV, bv)) return fail(DIRAC_EINVAL, "gV overlaps V or gW");
    rc = launch_links_backward(nc, g, V, gW, gV, as_stream(stream));
    if (rc) return fail(rc, "link backward launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

int dirac_project_su(const void* U, const void* g, void* F, int nc, int64_t nlinks, void* stream) {
    if (!U || !g || !F) return fail(DIRAC_EINVAL, "NULL pointer");
    if (nc < 1 || nc > 4) return fail(DIRAC_EUNSUPPORTED, "nc must be in 1..4");
    if (nlinks < 0) return fail(DIRAC_EINVAL, "negative link count");
    if (nlinks == 0) return DIRAC_OK;
    const size_t b = static_cast<size_t>(nlinks) * nc * nc * 16;
    if (overlap(U, b, F, b)) return fail(DIRAC_EINVAL, "F overlaps U");
    int rc = launch_project_su(nc, nlinks, U, g, F, as_stream(stream));
    if (rc) return fail(rc, "projection launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

static int blas_check(dirac_prec p, int64_t nrows, int nv) {
    if (p < DIRAC_FP64 || p > DIRAC_BF16) return fail(DIRAC_EINVAL, "unknown precision");
    if (nv < 1 || nv > 256) return fail(DIRAC_EINVAL, "nv must be in 1..256");
    if (nrows < 0) return fail(DIRAC_EINVAL, "negative row count");
    return DIRAC_OK;
}

size_t dirac_blas_workspace_bytes(int nv) {
    return (nv < 1 || nv > 256) ? 0 : reduce_partial_doubles(nv) * sizeof(double);
}

int dirac_norm2(dirac_prec prec, const void* x, int64_t nrows, int nv, double* out, void* workspace, size_t ws_bytes,
                void* stream) {
    int rc = blas_check(prec, nrows, nv);
    if (rc) return rc;
    if (!x || !out || !workspace) return fail(DIRAC_EINVAL, "NULL pointer");
    if (ws_bytes < dirac_blas_workspace_bytes(nv)) return fail(DIRAC_EWORKSPACE, "BLAS workspace too small");
    rc = blas_norm2(prec, x, nrows, nv, static_cast<double*>(workspace), out, as_stream(stream));
    if (rc) return fail(rc, "norm launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

int dirac_dot(dirac_prec prec_x, const void* x, dirac_prec prec_y, const void* y, int64_t nrows, int nv, double* out,
              void* workspace, size_t ws_bytes, void* stream) {
    int rc = blas_check(prec_x, nrows, nv);
    if (!rc) rc = blas_check(prec_y, nrows, nv);
    if (rc) return rc;
    if (!x || !y || !out || !workspace) return fail(DIRAC_EINVAL, "NULL pointer");
    if (ws_bytes < dirac_blas_workspace_bytes(nv)) return fail(DIRAC_EWORKSPACE, "BLAS workspace too small");
    rc = blas_dot(prec_x, x, prec_y, y, nrows, nv, static_cast<double*>(workspace), out, as_stream(stream));
    if (rc) return fail(rc, "dot launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

int dirac_dot_noalloc(dirac_prec prec_x, const void* x, dirac_prec prec_y, const void* y, int64_t nrows, int nv,
                      double* out, void* stream) {
    int rc = blas_check(prec_x, nrows, nv);
    if (!rc) rc = blas_check(prec_y, nrows, nv);
    if (rc) return rc;
    if (!x || !y || !out) return fail(DIRAC_EINVAL, "NULL pointer");
    if (reduce_partial_doubles(nv) > static_scratch_doubles())
        return fail(DIRAC_EINVAL, "nv beyond the static scratch (at most 256 right-hand sides)");
    double* partial = nullptr;
    if ((rc = static_scratch(&partial))) return rc;
    // every block writes all of its partials before the finalize reads them: nothing to clear
    rc = blas_dot(prec_x, x, prec_y, y, nrows, nv, partial, out, as_stream(stream));
    if (rc) return fail(rc, "dot launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

int dirac_caxpy(dirac_prec prec_x, const void* x, dirac_prec prec_y, void* y, const double* a, int64_t nrows, int nv,
                void* stream) {
    int rc = blas_check(prec_x, nrows, nv);
    if (!rc) rc = blas_check(prec_y, nrows, nv);
    if (rc) return rc;
    if (!x || !y || !a) return fail(DIRAC_EINVAL, "NULL pointer");
    if (overlap(x, nrows * nv * complex_bytes(prec_x), y, nrows * nv * complex_bytes(prec_y)))
        return fail(DIRAC_EINVAL, "x and y overlap");
    rc = blas_caxpy(prec_x, x, prec_y, y, a, nrows, nv, as_stream(stream));
    if (rc) return fail(rc, "caxpy launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

int dirac_cxpay(dirac_prec prec_x, const void* x, dirac_prec prec_y, void* y, const double* a, int64_t nrows, int nv,
                void* stream) {
    int rc = blas_check(prec_x, nrows, nv);
    if (!rc) rc = blas_check(prec_y, nrows, nv);
    if (rc) return rc;
    if (!x || !y || !a) return fail(DIRAC_EINVAL, "NULL pointer");
    if (overlap(x, nrows * nv * complex_bytes(prec_x), y, nrows * nv * complex_bytes(prec_y)))
        return fail(DIRAC_EINVAL, "x and y overlap");
    rc = blas_cxpay(prec_x, x, prec_y, y, a, nrows, nv, as_stream(stream));
    if (rc) return fail(rc, "cxpay launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

int dirac_cast(dirac_prec prec_x, const void* x, dirac_prec prec_y, void* y, int64_t ncomplex, void* stream) {
    int rc = blas_check(prec_x, ncomplex, 1);
    if (!rc) rc = blas_check(prec_y, ncomplex, 1);
    if (rc) return rc;
    if (!x || !y) return fail(DIRAC_EINVAL, "NULL pointer");
    if (ncomplex == 0) return DIRAC_OK;
    if (overlap(x, ncomplex * complex_bytes(prec_x), y, ncomplex * complex_bytes(prec_y)))
        return fail(DIRAC_EINVAL, "x and y overlap");
    rc = blas_cast(prec_x, x, prec_y, y, ncomplex, as_stream(stream));
    if (rc) return fail(rc, "cast launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

int dirac_gamma5(dirac_op op, dirac_prec prec, const void* x, void* y, int nc, int nv, const dirac_dims* dims,
                 void* stream) {
    Geom g;
    int rc = check_common(op, prec, nc, nv, dims, g);
    if (rc) return rc;
    if (!x || !y) return fail(DIRAC_EINVAL, "NULL pointer");
    rc = blas_gamma5(op, prec, x, y, nc, nv, g, as_stream(stream));
    if (rc) return fail(rc, "gamma5 launch rejected");
    DIRAC_HIP(hipGetLastError());
    return DIRAC_OK;
}

size_t dirac_solver_workspace_bytes(dirac_op op, int solver, dirac_prec outer, dirac_prec inner, int nc, int nv,
                                    const dirac_dims* dims) {
    Geom g;
    if (check_common(op, outer, nc, nv, dims, g)) return 0;
    if (inner < DIRAC_FP64 || inner > DIRAC_BF16 || solver < 0 || solver > 1) return 0;
    // room for either mixed scheme
    const size_t a = solver_workspace_bytes(op, solver, outer, inner, nc, nv, g, 0);
    const size_t b = solver_workspace_bytes(op, solver, outer, inner, nc, nv, g, 1);
    return a > b ? a : b;
}

static int solve(int solver, dirac_op op, dirac_prec outer, dirac_prec inner, const void* gauge_hi,
                 const void* gauge_lo, const void* b, void* x, double mass, int nc, int nv, const dirac_dims* dims,
                 double tol, int maxit, void* workspace, size_t ws_bytes, dirac_solve_info* info,
                 const dirac_solve_opts* opts, void* stream) {
    Geom g;
    int rc = check_common(op, outer, nc, nv, dims, g);
    if (rc) return rc;
    if (outer == DIRAC_BF16) return fail(DIRAC_EUNSUPPORTED, "outer precision must be FP64 or FP32");
    if (inner < DIRAC_FP64 || inner > DIRAC_BF16) return fail(DIRAC_EINVAL, "unknown inner precision");
    const bool mixed = inner != outer;
    if (mixed && (outer != DIRAC_FP64 || inner == DIRAC_FP64))
        return fail(DIRAC_EUNSUPPORTED, "mixed precision needs an FP64 outer and an FP32/BF16 inner precision");
    if (solver == 1 && op != DIRAC_WILSON && op != DIRAC_BRILLOUIN)
        return fail(DIRAC_EUNSUPPORTED, "BiCGstab is for Wilson and Brillouin");
    if (!gauge_hi || !b || !x || !workspace || (mixed && !gauge_lo)) return fail(DIRAC_EINVAL, "NULL pointer");
    const void* clov_hi = opts ? opts->clover_hi : nullptr;
    const void* clov_lo = opts ? opts->clover_lo : nullptr;
    if (clov_hi) {
        if (!op_takes_clover(op)) return fail(DIRAC_EINVAL, "the clover term belongs to Wilson and Brillouin");
        if (mixed && !clov_lo) return fail(DIRAC_EINVAL, "a mixed solve with a clover field needs clover_lo");
        if (!aligned(clov_hi, outer == DIRAC_FP64 ? 8 : 4) || (mixed && !aligned(clov_lo, 4)))
            return fail(DIRAC_EINVAL, "misaligned clover field");
    }
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(DIRAC_EINVAL, "tolerance must be positive");
    if (maxit < 0) return fail(DIRAC_EINVAL, "maxit must be >= 0");
    if (!std::isfinite(mass)) return fail(DIRAC_EINVAL, "mass is not finite");
    const size_t vb = static_cast<size_t>(rows_of(op, nc, g)) * nv * complex_bytes(outer);
    if (overlap(b, vb, x, vb)) return fail(DIRAC_EINVAL, "b and x overlap");
    if (overlap(workspace, ws_bytes, x, vb) || overlap(workspace, ws_bytes, b, vb))
        return fail(DIRAC_EINVAL, "workspace overlaps b or x");
    if (info) {
        info->iters = info->outer_iters = info->reason = 0;
        info->hist_len = 0;
    }
    return run_solver(solver, op, outer, inner, gauge_hi, gauge_lo, clov_hi, mixed ? clov_lo : nullptr, b, x, mass,
                      nc, nv, g, tol, maxit, workspace, ws_bytes, info, opts, as_stream(stream));
}

int cg_solve(dirac_op op, dirac_prec outer, dirac_prec inner, const void* gauge_hi, const void* gauge_lo,
             const void* b, void* x, double mass, int nc, int nv, const dirac_dims* dims, double tol, int maxit,
             void* workspace, size_t ws_bytes, dirac_solve_info* info, const dirac_solve_opts* opts, void* stream) {
    return solve(0, op, outer, inner, gauge_hi, gauge_lo, b, x, mass, nc, nv, dims, tol, maxit, workspace, ws_bytes,
                 info, opts, stream);
}

int bicgstab_solve(dirac_op op, dirac_prec outer, dirac_prec inner, const void* gauge_hi, const void* gauge_lo,
                   const void* b, void* x, double mass, int nc, int nv, const dirac_dims* dims, double tol, int maxit,
                   void* workspace, size_t ws_bytes, dirac_solve_info* info, const dirac_solve_opts* opts,
                   void* stream) {
    return solve(1, op, outer, inner, gauge_hi, gauge_lo, b, x, mass, nc, nv, dims, tol, maxit, workspace, ws_bytes,
                 info, opts, stream);
}

int dirac_set_launch_shape(dirac_op op, dirac_prec prec, int rb, int variant) {
    if (op < DIRAC_WILSON || op > DIRAC_BRILLOUIN_LAPLACE || prec < DIRAC_FP64 || prec > DIRAC_BF16)
        return fail(DIRAC_EINVAL, "unknown operator or precision");
    const int maxrb = op_uses_w(op) ? 1 : (op == DIRAC_WILSON ? 2 : 4);
    if (rb != 0 && rb != 1 && rb != 2 && rb != 4) return fail(DIRAC_EINVAL, "rb must be 0, 1, 2 or 4");
    if (rb > maxrb) return fail(DIRAC_EUNSUPPORTED, "rb not instantiated for this operator");
    if (variant != 0 && variant != 1 && variant != 4) return fail(DIRAC_EINVAL, "variant must be 0, 1 or 4");
    g_rb_override[op][prec] = rb;
    g_variant_override[op][prec] = variant;
    return DIRAC_OK;
}

double dirac_flops_per_site(dirac_op op, int nc) {
    const double n = nc;
    switch (op) {
        case DIRAC_WILSON: return 128.0 * n * n + 72.0 * n;
        case DIRAC_BRILLOUIN: return 2560.0 * n * n + 2376.0 * n;
        case DIRAC_STAGGERED: return 64.0 * n * n + 2.0 * n;
        case DIRAC_WILSON_LAPLACE: return 256.0 * n * n + 8.0 * n;
        case DIRAC_BRILLOUIN_LAPLACE: return 2560.0 * n * n + 648.0 * n;
    }
    return 0.0;
}

const char* dirac_error_string(int status) {
    switch (status) {
        case DIRAC_OK: return "ok";
        case DIRAC_NOT_CONVERGED: return "solver did not converge (iteration limit or stagnation)";
        case DIRAC_EINVAL: return "invalid argument";
        case DIRAC_EUNSUPPORTED: return "unsupported configuration";
        case DIRAC_EHIP: return "HIP runtime error";
        case DIRAC_EWORKSPACE: return "workspace too small";
        case DIRAC_ENONFINITE: return "non-finite value in a norm";
    }
    return "unknown status";
}

const char* dirac_last_error(void) { return g_last_error.c_str(); }

const char* dirac_version(void) { return "libdirac 0.1 (gfx950)"; }

}  // extern "C"
