// Internal launcher interface between the C ABI / solvers and the kernel files.
#pragma once

#include "common.h"

namespace dirac {

// Solver epilogue of a row-tiled stencil launch (Wilson, staggered; the CG iteration on D^+ D):
//   mode 1: the output is written as usual and each tile also writes the per-RHS sums of |out|^2 of its
//           sites (values as stored) to partial[tile * nv + rhs];
//   mode 2: the output q is not written: r -= alpha q (alpha: 2 nv doubles, complex, device; q as it would
//           have been stored; r in FP64 for FP64 applies, FP32 otherwise) and the tile writes the per-RHS
//           sums of |r|^2 (r as stored) to partial[tile * nv + rhs].
// Tiles are x-rows: V / N_x of them.
struct Epilogue {
    int mode = 0;
    double* partial = nullptr;
    void* r = nullptr;
    const double* alpha = nullptr;
};

struct StencilArgs {
    dirac_prec prec;
    int nc;
    int nv;
    int rb;       // right-hand sides per thread (divides the columns the kernel sees)
    int variant;  // 1: direct global loads, 4: row tiles staged in LDS (falls back to 1 where a row does not fit)
    bool dagger;
    double mass;
    Geom g;
    const void* gauge;
    const void* in;
    void* out;
    const void* clover = nullptr;  // packed clover blocks (clover.h) for Wilson / Brillouin, or none
    bool laplace = false;          // the spin-trivial Laplace operator of the same stencil
    Epilogue epi;                  // solver epilogue (row tiles of Wilson and staggered only)
};

// Return value of the launchers when an epilogue was asked for but the launch shape cannot apply it
// (nothing was launched; the caller runs the unfused sequence).
constexpr int kNoEpilogue = 100;

// Stencil launches (asynchronous; arguments already validated).
int launch_wilson(const StencilArgs& a, hipStream_t st);
int launch_staggered(const StencilArgs& a, hipStream_t st);
int launch_brillouin(const StencilArgs& a, hipStream_t st);
int launch_brillouin_links(dirac_prec prec, int nc, const Geom& g, const void* U, void* W, hipStream_t st);
int launch_clover_field(dirac_prec prec, int nc, const Geom& g, const void* U, void* C, double csw, hipStream_t st);
size_t clover_field_reals(int nc);

// Operator classes.  The Laplace operators act on Wilson-layout vectors ([colour][spin][rhs]) and are
// hermitian; they run on the staggered (Wilson Laplacian) and Brillouin (Brillouin Laplacian) kernels.
inline bool op_is_laplace(dirac_op op) { return op == DIRAC_WILSON_LAPLACE || op == DIRAC_BRILLOUIN_LAPLACE; }
inline bool op_four_spin(dirac_op op) { return op != DIRAC_STAGGERED; }
inline bool op_uses_w(dirac_op op) { return op == DIRAC_BRILLOUIN || op == DIRAC_BRILLOUIN_LAPLACE; }
inline bool op_takes_clover(dirac_op op) { return op == DIRAC_WILSON || op == DIRAC_BRILLOUIN; }

// Launch one apply of `op` (D, D^+ with dag; the Laplacians ignore dag); rb and variant from the defaults
// or the dirac_set_launch_shape overrides.
int launch_stencil(dirac_op op, dirac_prec prec, int nc, int nv, const Geom& g, double mass, const void* gauge,
                   const void* clover, const void* in, void* out, bool dag, hipStream_t st,
                   const Epilogue& epi = Epilogue());
int launch_force(dirac_op op, int nc, int nv, const Geom& g, const void* U, const void* psi, const void* chi,
                 void* gout, double coeff, hipStream_t st);
int launch_project_su(int nc, int64_t nlinks, const void* U, const void* g, void* F, hipStream_t st);
int launch_stout(int nc, const Geom& g, const void* U, void* V, double rho, hipStream_t st);
int launch_stout_backward(int nc, const Geom& g, const void* U, const void* gV, void* gU, double rho, hipStream_t st);
int launch_links_backward(int nc, const Geom& g, const void* V, const void* gW, void* gV, hipStream_t st);

// RHS-per-thread choice for a stencil (tunable; divides the columns the kernel sees) and kernel variant.
int choose_rb(dirac_op op, dirac_prec prec, int nc, int nv, const Geom& g);
int choose_variant(dirac_op op, dirac_prec prec);

// ---------------------------------------------------------------------------
// Multi-RHS BLAS-1.  Rows of nv complex numbers, rhs fastest.  Reductions are two-pass
// with a fixed number of blocks and a fixed summation order; `partial` must hold
// reduce_partial_doubles(nv) doubles of device scratch.
// ---------------------------------------------------------------------------
constexpr int kReduceBlocks = 2048;
constexpr int kReduceThreads = 256;
inline size_t reduce_partial_doubles(int nv) { return static_cast<size_t>(kReduceBlocks) * 2 * nv; }

int blas_norm2(dirac_prec p, const void* x, int64_t nrows, int nv, double* partial, double* out, hipStream_t st);
// out[rhs] = sum over nblk blocks of partial[b * nv + rhs] (fixed order), e.g. the per-tile partials
// of a stencil epilogue; scratch: 256 * nv doubles of device memory
void finalize_blocks(const double* partial, int64_t nblk, int nv, double* scratch, double* out, hipStream_t st);
// Device address of the library's own reduction partials on the current device (found once per
// device); static_scratch_doubles() doubles, enough for reduce_partial_doubles(256).
int static_scratch(double** out);
size_t static_scratch_doubles();
int blas_dot(dirac_prec px, const void* x, dirac_prec py, const void* y, int64_t nrows, int nv, double* partial,
             double* out, hipStream_t st);
// y += a x  (a: device, 2 nv doubles)
int blas_caxpy(dirac_prec px, const void* x, dirac_prec py, void* y, const double* a, int64_t nrows, int nv,
               hipStream_t st);
// y = x + a y
int blas_cxpay(dirac_prec px, const void* x, dirac_prec py, void* y, const double* a, int64_t nrows, int nv,
               hipStream_t st);
int blas_cast(dirac_prec px, const void* x, dirac_prec py, void* y, int64_t ncomplex, hipStream_t st);
int blas_gamma5(dirac_op op, dirac_prec p, const void* x, void* y, int nc, int nv, const Geom& g, hipStream_t st);
// y = x * s_i, s real per RHS (device, nv doubles)
int blas_rscale(dirac_prec px, const void* x, dirac_prec py, void* y, const double* s, int64_t nrows, int nv,
                hipStream_t st);

// Fused solver kernels (see solvers.cpp for their role).
// r -= alpha q ; out(rr) = ||r||^2   (alpha: device 2nv doubles; r, q same precision p)
int fused_r_update(dirac_prec pr, void* r, dirac_prec pq, const void* q, const double* alpha, int64_t nrows, int nv,
                   double* partial, double* rr, hipStream_t st);
// x += alpha p ; p = r + beta p   (x precision px; r, p precision pp)
int fused_xp_update(dirac_prec px, void* x, dirac_prec pp, void* p, dirac_prec prr, const void* r, const double* alpha,
                    const double* beta, int64_t nrows, int nv, hipStream_t st);
// x += alpha p ; p = r + beta p ; rp = <r, p> of the new p as stored (2 nv doubles, re/im per RHS).
// With `burst` (device, burst_partial_doubles(nrows, nv) doubles, may be null) each thread takes a few
// rows once, all loads first, and the per-block partials are summed in two fixed-order stages.
size_t burst_partial_doubles(int64_t nrows, int nv);
int fused_xp_update_dot(dirac_prec px, void* x, dirac_prec pp, void* p, dirac_prec prr, const void* r,
                        const double* alpha, const double* beta, int64_t nrows, int nv, double* partial, double* rp,
                        hipStream_t st, double* burst = nullptr, size_t burst_doubles = 0);
// y = b - y  (residual from A x stored in y)
int blas_bminus(dirac_prec pb, const void* b, dirac_prec py, void* y, int64_t nrows, int nv, hipStream_t st);
// r = b - q (all complex elements, any precisions)
int blas_sub(dirac_prec pb, const void* b, dirac_prec pq, const void* q, dirac_prec pr, void* r, int64_t n,
             hipStream_t st);
// BiCGstab: x += alpha p + omega s ; r = s - omega t ; out = ||r||^2
int fused_bicg_xr(dirac_prec p, void* x, const void* pv, const void* s, const void* t, void* r, const double* alpha,
                  const double* omega, int64_t nrows, int nv, double* partial, double* rr, hipStream_t st);
// BiCGstab: p = r + beta (p - omega v)
int fused_bicg_p(dirac_prec p, void* pv, const void* r, const void* v, const double* beta, const double* omega,
                 int64_t nrows, int nv, hipStream_t st);
// BiCGstab: s = r - alpha v
int fused_bicg_s(dirac_prec p, void* s, const void* r, const void* v, const double* alpha, int64_t nrows, int nv,
                 hipStream_t st);

}  // namespace dirac
