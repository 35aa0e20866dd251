/*
 * dirac.h -- C ABI of libdirac, the MI355X (gfx950) implementation of the
 * multi-right-hand-side Dirac-operator hot path of Duerr, "Fast and flexible
 * implementations of Wilson, Brillouin and Susskind fermions in lattice QCD"
 * (arXiv:2112.14640).
 *
 * General rules for every entry point
 * -----------------------------------
 * - Every array argument is a DEVICE pointer owned by the caller.  The library
 *   never frees caller memory and allocates no device memory in the apply,
 *   link, force, projection and BLAS-1 calls; solvers use only the workspace the
 *   caller passes (size from dirac_solver_workspace_bytes).
 * - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL is
 *   the null stream), except the solvers, which synchronise `stream` once per
 *   iteration to read the per-RHS residual norms, and return after the solve.
 * - Every call returns an int status (below) and never throws or aborts.
 *   Arguments are validated before any launch; on error nothing is launched
 *   and dirac_last_error() returns a description.
 * - Complex numbers are interleaved (re, im).  FP64 = complex128 (2 doubles),
 *   FP32 = complex64 (2 floats), BF16 = 2 bfloat16 (re, im), rounded to nearest
 *   even on every store.
 *
 * Lattice and layouts
 * -------------------
 * Site n = (x, y, z, t), 0-based; linear site index s = ((t*Nz + z)*Ny + y)*Nx + x.
 * Direction mu = 0,1,2,3 is x,y,z,t.  Links are periodic; fermion fields are
 * periodic in x,y,z and, if dims->antiperiodic_t is set, antiperiodic in t
 * (a hop that wraps in t multiplies the fetched spinor by -1).
 *   gauge U   : [s][mu][a][b]           U_mu(n), row a, column b; transports n+mu -> n
 *   links W   : [s][dir][a][b]          40 stored Brillouin links (see dirac_brillouin_links)
 *   Wilson/Brillouin vector : [s][colour][spin][rhs]  (Nc x 4 x Nv complex per site, rhs fastest)
 *   staggered vector        : [s][colour][rhs]        (Nc x Nv complex per site)
 * Gamma matrices are the chiral basis of App. A of the paper.
 */
#ifndef DIRAC_H
#define DIRAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define DIRAC_OK 0
#define DIRAC_NOT_CONVERGED 1   /* solver: iteration limit or stagnation; x holds the last iterate */
#define DIRAC_EINVAL (-1)       /* bad op/prec/extent/pointer/alias/size */
#define DIRAC_EUNSUPPORTED (-2) /* colour count or precision combination not instantiated */
#define DIRAC_EHIP (-3)         /* HIP runtime error (details in dirac_last_error) */
#define DIRAC_EWORKSPACE (-4)   /* solver workspace too small */
#define DIRAC_ENONFINITE (-5)   /* non-finite norm of b or of a residual */

/* Operators.  The two Laplace operators are the spin-trivial "embedded" Laplacians of Secs. 5 and 6,
 * acting on Wilson-layout vectors; they are hermitian (D^dagger = D). */
typedef enum {
    DIRAC_WILSON = 0,
    DIRAC_BRILLOUIN = 1,
    DIRAC_STAGGERED = 2,
    DIRAC_WILSON_LAPLACE = 3,    /* -1/2 Delta^std + m^2/2 (Eq. app_wlap), gauge U */
    DIRAC_BRILLOUIN_LAPLACE = 4  /* -1/2 Delta^bri + m^2/2 (Eq. app_blap), gauge W */
} dirac_op;

/* Storage precision of the vectors.  FP64: complex128 vectors and complex128
 * gauge/links.  FP32: complex64 vectors and links.  BF16: bfloat16-pair vectors
 * with complex64 (FP32) gauge/links; arithmetic in FP32. */
typedef enum { DIRAC_FP64 = 0, DIRAC_FP32 = 1, DIRAC_BF16 = 2 } dirac_prec;

typedef struct {
    int32_t n[4];           /* Nx, Ny, Nz, Nt; each >= 2 (staggered: even) */
    int32_t antiperiodic_t; /* 1: fermion sign -1 on t-wrapping hops; 0: periodic */
} dirac_dims;

/* Supported colour counts: Nc in {1, 2, 3, 4}.  Nv (RHS count): 1..256. */

/*
 * v = D u.
 * Wilson (Sec. 5, Eq. app_wils, r = 1, c_SW = 0):
 *   (D_W u)(n) = (4+m) u(n) + 1/2 sum_mu {[(g_mu - 1) x U_mu(n)] u(n+mu) - [(g_mu + 1) x U_mu(n-mu)^+] u(n-mu)}
 * Brillouin (Sec. 6, Eqs. def_bril/def_ider/def_blap): 81-point hypercube stencil
 *   (D_B u)(n) = (m + 15/8) u(n) + sum_{d != 0} [(rho_|d| sum_mu d_mu g_mu - lambda_|d|/2) x W_d(n)] u(n+d)
 *   rho = (64,16,4,1)/432, lambda = (-240,8,4,2,1)/64; `gauge` is the stored link array W.
 * Staggered (Sec. 7, Eq. def_stag):
 *   (D_S u)(n) = m u(n) + 1/2 sum_mu eta_mu(n) [U_mu(n) u(n+mu) - U_mu(n-mu)^+ u(n-mu)],
 *   eta_mu(n) = (-1)^(x_0 + ... + x_{mu-1}) on 0-based coordinates.
 * Wilson Laplacian (Sec. 5, Eq. app_wlap; colour only, every spin component alike):
 *   (4 + m^2/2) u(n) - 1/2 sum_mu [U_mu(n) u(n+mu) + U_mu(n-mu)^+ u(n-mu)]
 * Brillouin Laplacian (Sec. 6, Eq. app_blap):
 *   (m^2/2 - lambda_0/2) u(n) - sum_{d != 0} (lambda_|d|/2) W_d(n) u(n+d)
 * gauge: U (Wilson, staggered, Wilson Laplacian) or W (Brillouin, Brillouin Laplacian) in the gauge
 * precision of `prec`.  Vectors: staggered layout for DIRAC_STAGGERED, Wilson layout for the others.
 * u, v : vectors in the layout of `op`; u and v must not overlap.
 * Errors: EINVAL (nulls, u == v, bad extents, nv out of range), EUNSUPPORTED (nc), EHIP.
 */
int dirac_apply(dirac_op op, dirac_prec prec, const void* gauge, const void* u, void* v, double mass, int nc,
                int nv, const dirac_dims* dims, void* stream);

/* v = D^dagger u: gamma_5 D gamma_5 for Wilson and Brillouin (Sec. 9: D is gamma_5-hermitian),
 * m - (hopping part) for staggered, D itself for the (hermitian) Laplacians.  Same arguments and
 * errors as dirac_apply. */
int dirac_apply_dagger(dirac_op op, dirac_prec prec, const void* gauge, const void* u, void* v, double mass,
                       int nc, int nv, const dirac_dims* dims, void* stream);

/* v = D^dagger D u through the caller's scratch vector tmp (App. F: the normal
 * operators of the CG solvers).  u, v, tmp pairwise distinct.  For the Laplacians (hermitian
 * positive definite, solved by CG directly) v = D u and tmp is not touched. */
int dirac_apply_normal(dirac_op op, dirac_prec prec, const void* gauge, const void* u, void* v, void* tmp,
                       double mass, int nc, int nv, const dirac_dims* dims, void* stream);

/*
 * Clover term (Sec. 4, Eq. def_clov): C(n) = -(c_SW/2) sum_{mu<nu} sigma_{mu nu} F_{mu nu}(n), sigma of
 * App. A, F_{mu nu}(n) the clover-leaf field strength (Q - Q^+)/(8i) with its trace removed, Q the sum of
 * the four plaquettes of the (mu, nu) plane that start and end at n.
 * dirac_clover_field builds the site-diagonal C once per gauge field: in the chiral basis C is two
 * hermitian 2Nc x 2Nc blocks per site (spins 0,1 and spins 2,3), stored packed as reals: per site block 0
 * then block 1, each the 2Nc diagonal entries followed by the entries (i, j), i < j, row by row as
 * (re, im); component i of a block is spin 2h + i/Nc, colour i%Nc.  c_SW is folded in.
 *   prec FP64: U complex128, clover doubles; FP32 or BF16: U complex64, clover floats.
 *   clover holds dirac_clover_field_bytes(prec, nc, dims) bytes (8 Nc^2 reals per site); it must not
 *   overlap U.  Errors: EINVAL, EUNSUPPORTED (nc), EHIP.
 * dirac_apply_clover / dirac_apply_clover_dagger: v = (D + C) u and v = (D + C)^dagger u = D^dagger u + C u
 *   (C is hermitian) for op DIRAC_WILSON or DIRAC_BRILLOUIN (Eqs. def_wils, def_bril with c_SW > 0);
 *   otherwise as dirac_apply.  clover comes from dirac_clover_field in the precision of `prec`.
 */
size_t dirac_clover_field_bytes(dirac_prec prec, int nc, const dirac_dims* dims);
int dirac_clover_field(dirac_prec prec, const void* U, double csw, void* clover, int nc, const dirac_dims* dims,
                       void* stream);
int dirac_apply_clover(dirac_op op, dirac_prec prec, const void* gauge, const void* clover, const void* u, void* v,
                       double mass, int nc, int nv, const dirac_dims* dims, void* stream);
int dirac_apply_clover_dagger(dirac_op op, dirac_prec prec, const void* gauge, const void* clover, const void* u,
                              void* v, double mass, int nc, int nv, const dirac_dims* dims, void* stream);

/*
 * Brillouin links (Sec. 6, Tab. off-axis): W_d(n) = average over all |d|! orderings of the
 * unit steps of d of the link products V_{s1}(n) V_{s2}(n+s1) ..., where a step -mu from x
 * uses V_mu(x-mu)^dagger.  Directions are numbered dir = 27(d_t+1)+9(d_z+1)+3(d_y+1)+(d_x+1);
 * the 40 directions dir < 40 are stored, W_d(n) for dir > 40 is W_{-d}(n+d)^dagger
 * (direction 80-dir at site n+d).  Computed in FP64.
 * prec: FP64 -> U, W complex128; FP32 or BF16 -> U, W complex64.
 * U: [s][4][nc][nc]; W: [s][40][nc][nc] (40*nc*nc complex per site).  U and W must not overlap.
 */
int dirac_brillouin_links(dirac_prec prec, const void* U, void* W, int nc, const dirac_dims* dims,
                          void* stream);

/*
 * Link gradient ("fermion force") of the bilinear Re sum_rhs psi^dagger D chi with
 * respect to the gauge field, in the convention g = dL/dRe U + i dL/dIm U:
 *   g += coeff * dRe(psi^+ D chi)/dU.
 * Wilson (from Eq. app_wils, the hops through U_mu(n)):
 *   g_mu(n) = -1/2 b sum_{s,rhs} [((1-g_mu) psi(n))_s chi_s(n+mu)^+ + chi_s(n) ((1+g_mu) psi(n+mu))_s^+]
 * Staggered (from Eq. def_stag): g_mu(n) = 1/2 eta_mu(n) b sum_rhs [psi(n) chi(n+mu)^+ - chi(n) psi(n+mu)^+]
 * Brillouin (from Eq. app_bril; the gradient with respect to the 40 stored links W, `U` is then W and g
 * has W's layout): g_d(n) = b sum_{s,rhs} [psi(n) (S_d chi(n+d))^+ + (psi(n+d) (S_{-d} chi(n))^+)^+],
 *   S_d = rho_|d| sum_mu d_mu g_mu - lambda_|d|/2 (W_d(n) also enters the hop n+d -> n as W_{-d}(n+d)^+).
 * (b = boundary sign of the hop).  FP64 only: U, psi, chi, g complex128; g has the gauge
 * layout and is accumulated into (the caller zeroes it first).  The clover term's gradient is not provided.
 */
int dirac_force(dirac_op op, const void* U, const void* psi, const void* chi, void* g, double coeff, int nc,
                int nv, const dirac_dims* dims, void* stream);

/*
 * Stout smearing (Sec. 2: the smeared links V of the operators; Morningstar and Peardon), one step:
 *   C_mu(n) = rho sum_{nu != mu} [U_nu(n) U_mu(n+nu) U_nu(n+mu)^+ + U_nu(n-nu)^+ U_mu(n-nu) U_nu(n-nu+mu)],
 *   Omega = C U^+, Q = (i/2)(Omega^+ - Omega) - (i/(2Nc)) Tr(Omega^+ - Omega), V_mu(n) = exp(i Q) U_mu(n),
 * all links from the old field (the paper's default is three steps of rho = 0.12; call once per step).
 * dirac_stout_backward: gU += dL/dU for L(V(U)) given gV = dL/dV (one step; U is that step's input).
 * dirac_brillouin_links_backward: gV += dL/dV for L(W(V)) given gW = dL/dW on the 40 stored directions of
 *   dirac_brillouin_links (Tab. off-axis: path averages of V).
 * FP64 only: U, V, gU, gV complex128 [s][4][nc][nc]; gW complex128 [s][40][nc][nc].  Outputs must not overlap
 * the inputs.  The backward calls add with atomics: the summation order, and so the last bits, can vary
 * from run to run.  Errors: EINVAL, EUNSUPPORTED (nc), EHIP.
 */
int dirac_stout_smear(const void* U, void* V, double rho, int nc, const dirac_dims* dims, void* stream);
int dirac_stout_backward(const void* U, const void* gV, void* gU, double rho, int nc, const dirac_dims* dims,
                         void* stream);
int dirac_brillouin_links_backward(const void* V, const void* gW, void* gV, int nc, const dirac_dims* dims,
                                   void* stream);

/* su(Nc) projection of a link gradient: F = (i/2)(U g^+ - g U^+) minus trace/Nc, so that
 * dL/deps = sum tr(H F) for U -> exp(i eps H) U.  FP64; U, g, F: nlinks Nc x Nc matrices.
 * F may alias g. */
int dirac_project_su(const void* U, const void* g, void* F, int nc, int64_t nlinks, void* stream);

/*
 * Multi-RHS BLAS-1 (Sec. 3).  Vectors are `nrows` rows of `nv` complex (rhs fastest):
 * nrows = V*Nc*4 (Wilson/Brillouin) or V*Nc (staggered).  Reductions accumulate in FP64
 * with a fixed summation order (run-to-run bitwise reproducible), write to DEVICE arrays
 * of doubles and use the caller's device workspace of dirac_blas_workspace_bytes(nv) bytes
 * (returns 0 for an invalid nv).
 *   dirac_norm2: out[i] = ||x_i||^2                                    (nv doubles)
 *   dirac_dot  : out[2i], out[2i+1] = Re, Im <x_i, y_i> = sum conj(x) y (2 nv doubles;
 *                linear in the second argument, Sec. 3)
 *   dirac_caxpy: y_i += a_i x_i  (the paper's "incr", Eq. def_incr); a = 2 nv doubles (re, im), device
 *   dirac_cxpay: y_i = x_i + a_i y_i (the paper's "anti", Eq. def_anti)
 *   dirac_cast : y = x converted between precisions (BF16 stores round to nearest even)
 *   dirac_gamma5: y = gamma_5 x (Wilson layout) or y = epsilon x, epsilon = (-1)^(x+y+z+t)
 *                 (staggered layout) (Sec. 3); x may equal y
 * x and y may have different precisions in caxpy/cxpay/cast/dot (prec_x, prec_y); apart
 * from gamma5 they must not overlap.  Arithmetic is FP64.
 */
size_t dirac_blas_workspace_bytes(int nv);
int dirac_norm2(dirac_prec prec, const void* x, int64_t nrows, int nv, double* out, void* workspace, size_t ws_bytes,
                void* stream);
int dirac_dot(dirac_prec prec_x, const void* x, dirac_prec prec_y, const void* y, int64_t nrows, int nv, double* out,
              void* workspace, size_t ws_bytes, void* stream);
/* dirac_dot without a workspace argument, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The reduction partials live
 * in a library-owned device array of 8 MiB (2048 blocks x 2 x 256 doubles) that each GPU the library
 * runs on holds until the process ends; the call itself allocates nothing.  nv must be in 1..256
 * (EINVAL beyond).  The array is shared by every call on that GPU: calls that overlap in time on one GPU
 * (other streams, other threads) race and give wrong results; serialise them.  Same arguments,
 * results (bit for bit) and errors as dirac_dot otherwise. */
int dirac_dot_noalloc(dirac_prec prec_x, const void* x, dirac_prec prec_y, const void* y, int64_t nrows, int nv,
                      double* out, void* stream);
int dirac_caxpy(dirac_prec prec_x, const void* x, dirac_prec prec_y, void* y, const double* a, int64_t nrows,
                int nv, void* stream);
int dirac_cxpay(dirac_prec prec_x, const void* x, dirac_prec prec_y, void* y, const double* a, int64_t nrows,
                int nv, void* stream);
int dirac_cast(dirac_prec prec_x, const void* x, dirac_prec prec_y, void* y, int64_t ncomplex, void* stream);
int dirac_gamma5(dirac_op op, dirac_prec prec, const void* x, void* y, int nc, int nv, const dirac_dims* dims,
                 void* stream);

/*
 * Solvers (Sec. 9).  N_v independent solves in lock-step.
 *   cg_solve      : D^dagger D x = b   (conjugate gradients on the hermitian positive normal operator;
 *                                       for the two Laplacians, which are hermitian positive definite,
 *                                       D x = b directly)
 *   bicgstab_solve: D x = b            (BiCGstab; Wilson and Brillouin)
 * With opts->clover_hi (and clover_lo for a mixed solve) D is D + C (Wilson, Brillouin).
 * outer: precision of b and x (FP64 or FP32).  inner == outer: plain solve.  inner lower
 * than outer (FP32 or BF16 under an FP64 outer): mixed precision -- the true residual,
 * the solution update and all dot products stay in FP64 on the GPU while the operator
 * runs in the inner precision (see dirac_solve_opts.mixed_scheme).
 * gauge_hi: gauge (or W) in the outer gauge precision; gauge_lo: in the inner gauge
 * precision (complex64 for FP32/BF16); ignored (may be NULL) for plain solves.
 * x: initial guess on entry (zero it for a cold start), solution on return.
 * Stopping rule: ||b_i - A x_i|| <= tol ||b_i|| for every RHS, with the residual recomputed
 * explicitly (Sec. 9): recompute every `recompute_every` iterations (default 50 in FP64,
 * 20 in FP32/BF16), when the updated residuals suggest convergence, and at maxit; exit
 * when converged, when updated and recomputed norms differ by more than `drift`
 * (default 1 %), or at maxit.  A converged RHS is frozen.
 * workspace: device memory of at least dirac_solver_workspace_bytes(...) bytes.
 * info (optional, host): filled on return.  opts (optional, host): NULL for defaults.
 * Returns OK, NOT_CONVERGED, or an error (EINVAL, EUNSUPPORTED, EWORKSPACE, ENONFINITE, EHIP).
 */
typedef struct {
    int iters;            /* operator iterations (inner iterations for mixed solves) */
    int outer_iters;      /* residual recomputations in the outer precision */
    int reason;           /* 0 converged, 1 stagnated (drift), 2 iteration limit */
    double* true_relres;  /* host array [nv] or NULL: final ||b - A x|| / ||b|| per RHS (outer precision) */
    double* alpha;        /* host [hist_cap * nv] or NULL: CG step lengths, iteration-major (plain CG only) */
    double* beta;         /* host [hist_cap * nv] or NULL: CG direction ratios */
    int hist_cap;         /* capacity of alpha/beta in iterations */
    int hist_len;         /* number of iterations written */
} dirac_solve_info;

typedef struct {
    int recompute_every;  /* 0: default (50 FP64, 20 lower) */
    double drift;         /* 0: default 0.01 */
    int mixed_scheme;     /* 0: reliable updates (default), 1: defect correction (restarted inner solves) */
    double delta;         /* reliable-update factor (0: default 0.1); with defect correction the inner
                           * solves' relative tolerance (0: default 1e-5 FP32, 5e-2 BF16) */
    int max_outer;        /* defect-correction cycles; 0: default 100 */
    const void* clover_hi; /* clover field in the outer precision (dirac_clover_field) or NULL: no clover */
    const void* clover_lo; /* clover field in the inner precision (floats), needed by mixed solves with clover_hi */
} dirac_solve_opts;

size_t dirac_solver_workspace_bytes(dirac_op op, int solver /* 0 = CG on D^+D, 1 = BiCGstab on D */,
                                    dirac_prec outer, dirac_prec inner, int nc, int nv, const dirac_dims* dims);

int cg_solve(dirac_op op, dirac_prec outer, dirac_prec inner, const void* gauge_hi, const void* gauge_lo,
             const void* b, void* x, double mass, int nc, int nv, const dirac_dims* dims, double tol, int maxit,
             void* workspace, size_t ws_bytes, dirac_solve_info* info, const dirac_solve_opts* opts, void* stream);

int bicgstab_solve(dirac_op op, dirac_prec outer, dirac_prec inner, const void* gauge_hi, const void* gauge_lo,
                   const void* b, void* x, double mass, int nc, int nv, const dirac_dims* dims, double tol,
                   int maxit, void* workspace, size_t ws_bytes, dirac_solve_info* info,
                   const dirac_solve_opts* opts, void* stream);

/* Launch-shape knob for the stencil kernels of (op, prec): rb = right-hand-side columns handled by
 * one thread (0 automatic; Wilson 1 or 2, staggered and Wilson Laplacian 1, 2 or 4, Brillouin and
 * Brillouin Laplacian 1; used whenever it divides the columns; the Wilson Laplacian sees 4 Nv columns);
 * variant = 0 automatic, 1 direct global loads (one thread per site and rb columns), 4 row tiles
 * (a work-group stages one x-row of the lattice and its neighbour rows in LDS with contiguous loads,
 * the next row in flight while the current one is consumed; Wilson with Nv = 12 and staggered in
 * FP32/BF16 also stage each direction's links in LDS; the Brillouin kernels walk the 27 neighbouring
 * x-rows with a window of three links per site).  Row tiles fall back to direct loads for shapes they
 * cannot take.  Results agree to rounding whatever the shape.  Process-wide, not thread-safe. */
int dirac_set_launch_shape(dirac_op op, dirac_prec prec, int rb, int variant);

/* Flop count per site and RHS of one apply, App. E convention (daggers count the same). */
double dirac_flops_per_site(dirac_op op, int nc);

/* Static description of a status code; never NULL. */
const char* dirac_error_string(int status);
/* Detail of the last failing call on this host thread ("" if none). */
const char* dirac_last_error(void);
/* Library version string. */
const char* dirac_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DIRAC_H */
