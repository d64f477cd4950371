/*
 * th.h -- C ABI of the MI355X two-grid Helmholtz library.
 *
 * The library solves the finite-element Helmholtz problem
 *     -Laplace u - (k(x)^2 + i eps(x)) u = f      on the unit square (cube),
 * with absorbing (Robin, du/dn - i k u = 0) or Neumann sides (Sec. 2 of
 * Stolk, "A two-grid method with dispersion matching for finite-element
 * Helmholtz problems", arXiv 2509.17494, eq. Helmholtz_eq and eq. bilin_form),
 * discretised with continuous Q_p elements (p even) on N x N cells of size
 * h = 1/N (Sec. 3.1), and applies the paper's two-grid method (Alg. 1):
 * complex-shifted domain-decomposition smoothing (Alg. 2), a QSFEM
 * dispersion-minimising coarse operator on the mesh of spacing 2h/p
 * (Sec. 3.2-3.3) and Q_{p/2} interpolation between the levels (Sec. 4.2),
 * used as the preconditioner of an FP64 GMRES.
 *
 * Conventions for every call:
 *   - Every function returns th_status; nothing throws across the ABI.  On a
 *     failure th_last_error(ctx) holds a message until the next call on ctx.
 *   - Fine vectors have (pN+1)^d complex entries, one per GLL node of the
 *     global node grid, lexicographic with x fastest.  Coarse vectors have
 *     (pN/2+1)^d entries on the coarse vertex grid, x fastest.
 *   - Vector arguments are DEVICE pointers owned by the caller, holding
 *     nrhs vectors back to back (layout [nrhs][ndof]), complex interleaved
 *     (re, im): double pairs for TH_C128, float pairs for TH_C64.  The
 *     library never allocates, frees or retains caller buffers.
 *   - Work is ordered on the stream given to th_create (NULL = the default
 *     stream).  Calls marked "stream-ordered" return before the GPU has
 *     finished; th_setup_* and th_solve block until their work is done.
 *   - One context per host thread; a context is not thread safe.
 */
#ifndef TH_H
#define TH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct th_ctx th_ctx;

typedef enum {
  TH_OK = 0,
  TH_EINVAL = -1,        /* bad argument: shape, order, NULL pointer, NaN input */
  TH_ESTATE = -2,        /* call out of order (e.g. smooth before setup) */
  TH_ENOMEM = -3,        /* device allocation failed */
  TH_EHIP = -4,          /* HIP runtime error; message in th_last_error */
  TH_ENOTCONV = -5,      /* th_solve hit maxit; u holds the last iterate */
  TH_ENUMERIC = -6,      /* NaN/Inf met in a norm or a pivot */
  TH_EUNSUPPORTED = -7   /* valid request this build does not implement */
} th_status;

/* Boundary conditions per side (eq. Helmholtz_eq): absorbing du/dn - i k u = 0,
 * Neumann du/dn = 0, homogeneous Dirichlet u = 0.  The nodes of a closed
 * Dirichlet side are eliminated on the fine grid, on the coarse vertex grid,
 * in every subdomain matrix and from I_P; vectors keep full length and the
 * operators carry unit rows and columns there (th_residual returns f - u on
 * those nodes).  With f = 0 on them, every iterate of th_solve is 0 there. */
typedef enum { TH_BC_ROBIN = 0, TH_BC_NEUMANN = 1, TH_BC_DIRICHLET = 2 } th_bc;
typedef enum { TH_C128 = 0, TH_C64 = 1 } th_dtype;

/* Storage / arithmetic of the dense subdomain operators B_i.
 * F64: complex128.  F32: complex64.  BF16: planar (re, im) bfloat16 with
 * FP32 accumulation. */
typedef enum { TH_GEMM_F64 = 0, TH_GEMM_F32 = 1, TH_GEMM_BF16 = 2 } th_gemm;

typedef enum {
  TH_COARSE_QSFEM = 0,    /* per-cell QSFEM weights q(h_c k(c)), Sec. 3.3; in 3-D the
                             27-point stencil exact at k (see th_plain_fit3d) */
  TH_COARSE_PLAINFIT = 1, /* per-cell plain dispersion-matching fit (th_plain_fit, or
                             th_plain_fit3d in 3-D) */
  TH_COARSE_MLP = 2,      /* per-cell surrogate network with fallback to the plain fit
                             (network family matching the dimension) */
  TH_COARSE_WEIGHTS = 3   /* caller-supplied per-coarse-cell (q0, q_edge, q_diag), or
                             (q0, q_face, q_edge, q_corner) in 3-D; weights are on the
                             2-D element scale (symbol -eta^2 at 0), a 3-D cell
                             contributes h_c q */
} th_coarse_scheme;

typedef struct th_mlp th_mlp;

/* Outer iteration around the preconditioner f -> TwoGridStep(0, f) (Sec. 4,
 * Alg. 1).  The paper leaves the Krylov method open.  GMRES_RIGHT and FGMRES
 * run the same code: right-preconditioned GMRES from x0 = 0 that stores the
 * preconditioned directions z_j = B(v_j) and forms x = x0 + sum y_j z_j, which
 * is flexible GMRES (needed when the preconditioner runs in complex64 and
 * varies with rounding) and equals plain right-preconditioned GMRES for the
 * FP64 preconditioner. */
typedef enum {
  TH_KRYLOV_GMRES_RIGHT = 0,  /* right-preconditioned GMRES (preconditioned directions stored) */
  TH_KRYLOV_FGMRES = 1,       /* flexible GMRES: the same iteration */
  TH_KRYLOV_STATIONARY = 2    /* u <- TwoGridStep(u, f) repeated from u = 0 */
} th_krylov;

/* Layout of the FP64/FP32 subdomain solves (th_fine_desc.layout).
 *   DENSE:     B_i = diag(1/L_j) R_U (A_s^(i))^{-1}, n_U x n_Omega, 64-row blocks.
 *   SYMMETRIC: the same with the U x U block of the symmetric inverse stored once
 *              (upper 64 x 64 tiles).
 *   SLAB:      block factorisation of A_s^(i) over slabs of P node layers along
 *              the slowest axis (the inverses of its Schur blocks and the slab
 *              couplings), applied by forward and backward sweeps: far fewer
 *              bytes for large subdomains, two launches per slab.
 *   AUTO picks by modelled time (bytes over bandwidth plus launches). */
typedef enum {
  TH_LAYOUT_AUTO = 0, TH_LAYOUT_DENSE = 1, TH_LAYOUT_SYMMETRIC = 2, TH_LAYOUT_SLAB = 3
} th_layout;

/* Fine-level problem and smoother parameters (Sec. 2, 3.1, 4.1, 4.4). */
typedef struct {
  int dim;              /* 2 or 3 (3-D: orders 2 and 4) */
  int n;                /* cells per direction N >= 1 */
  int order;            /* p in {2, 4, 6, 8} */
  const double *k;      /* HOST, N^d per-cell wavenumbers > 0, x fastest; copied */
  const double *eps;    /* HOST, N^d per-cell damping >= 0, or NULL for 0; copied */
  int bc[6];            /* sides x-, x+, y-, y+, (z-, z+): th_bc */
  double alpha_s;       /* smoother shift: volume coefficient k^2 + i alpha_s k^2 + i eps */
  int l_dd;             /* subdomain size in cells (blocks of ceil(N / l_dd) per direction) */
  int n_dd;             /* DD iterations per smoother step (>= 1) */
  int n_s;              /* pre- and post-smoothing steps (>= 1) */
  double omega_c;       /* coarse-grid correction relaxation */
  th_gemm gemm;         /* storage of the subdomain operators */
  int max_rhs;          /* largest nrhs of any later call (sizes the workspaces) */
  th_layout layout;     /* FP64/FP32 storage layout of the subdomain solves (0 = automatic);
                           BF16 storage has the matrix-core layout only */
} th_fine_desc;

/* Direct solver of the coarse system (th_coarse_desc.solver).  Both are exact
 * FP64 factorisations computed once on the device at setup; they differ in
 * the order of elimination, hence in bytes streamed and launches per solve.
 * ND eliminates interior separator blocks that can be nearly singular (real
 * indefinite Helmholtz blocks), so setup adds iterative-refinement steps (up
 * to 3) until the probe solve is within 1e-13 for th_coarse_solve and
 * th_twogrid (th_info.coarse_refine_exact), within 1e-8 inside the FP64
 * preconditioner of th_solve (th_info.coarse_refine), where Sec. 1 allows an
 * approximate coarse solve and the true-residual stopping rule decides.
 *   LINES:  block elimination over super-blocks of grid lines (planes in 3-D),
 *           explicit inverses of the Schur blocks (twisted when the slab
 *           right-hand sides fit in LDS).
 *   ND:     nested dissection of the vertex grid by separator lines (planes),
 *           multifrontal elimination with explicit inverses of every
 *           separator's frontal block; two launches per tree level.
 *   AUTO:   ND, unless its modelled solve time (factor bytes over bandwidth
 *           and a latency per launch, for max_rhs right-hand sides) exceeds
 *           that of LINES, its setup runs out of memory or its probe check (a
 *           solve against A_c x for a vector of unit-modulus entries, reported
 *           in th_info.coarse_check) misses 1e-9; then LINES. */
typedef enum { TH_CSOLVE_AUTO = 0, TH_CSOLVE_LINES = 1, TH_CSOLVE_ND = 2 } th_coarse_solver;

typedef struct {
  th_coarse_scheme scheme;
  const double *q;      /* HOST, (pN/2)^d x 3 (2-D) or x 4 (3-D) weights, x fastest;
                           TH_COARSE_WEIGHTS only */
  const th_mlp *mlp;    /* trained surrogate; TH_COARSE_MLP only */
  double fallback_tau;  /* TH_COARSE_MLP: a cell falls back to the plain fit when the zero
                           set of the network's stencil lies farther than this (relative
                           to eta) from the fine dispersion curve anywhere in the sector of
                           wave directions (th_mlp_stencils); 0 = every cell falls back */
  th_coarse_solver solver; /* coarse factorisation (0 = automatic) */
} th_coarse_desc;

typedef struct {
  th_krylov krylov;
  double rtol;          /* per right-hand side, converged when the TRUE FP64 residual
                           satisfies ||f - A u||_2 / ||f||_2 <= rtol.  GMRES leaves a
                           cycle on its recurrence residual, then forms f - A u; a
                           right-hand side still above rtol restarts from it */
  int maxit;            /* two-grid preconditioner applications (iterations) per RHS */
  int restart;          /* GMRES cycle length; <= 0: no restart (the Krylov basis grows
                           in blocks of 8 vectors of max_rhs x n_fine as the iteration
                           reaches them) */
  th_dtype precond_dtype; /* TH_C128: FP64 preconditioner; TH_C64: complex64 */
  int use_graph;        /* 1: capture the two-grid preconditioner once in a HIP graph and
                           replay it every iteration (needs a non-NULL stream; ignored
                           while kernel timing is enabled) */
} th_solve_opts;

typedef struct {
  int iters;            /* largest iteration count over the RHS */
  double rel_res;       /* largest true relative residual ||f - A u|| / ||f|| (FP64) */
  double t_solve_s;     /* wall time of the solve */
  long long n_precond;  /* two-grid preconditioner applications (summed over RHS) */
  double t_cycle_s;     /* t_solve_s / iters: wall time of one iteration (one two-grid
                           cycle for all RHS with its matvec and orthogonalisation) */
  int n_fallback_cells; /* TH_COARSE_MLP: coarse cells that fell back to the plain fit */
} th_solve_stats;

typedef struct {
  long long n_fine;       /* (pN+1)^d */
  long long n_coarse;     /* (pN/2+1)^d */
  int n_sub;              /* number of subdomains */
  long long b_entries;    /* sum over subdomains of n_U * n_Omega */
  long long b_bytes;      /* device bytes of the stored subdomain operators */
  long long coarse_bytes; /* device bytes of the coarse factors */
  double t_setup_fine_s, t_setup_coarse_s;
  int smoother_cfg;       /* matrix-core smoother configuration chosen by the autotuner */
  int smoother_grid;      /* its persistent grid size (0: one workgroup per work item) */
  int coarse_lines;       /* grid lines (2-D) or planes (3-D) per coarse super-block */
  int n_fallback_cells;   /* TH_COARSE_MLP: coarse cells that fell back to the plain fit */
  double t_stencil_s;     /* time spent computing the per-cell coarse weights */
  int smoother_layout;    /* storage of the subdomain operators: 0 dense rows (FP64/FP32),
                             1 symmetric tiles (FP64/FP32; the U x U block of the symmetric
                             inverse stored once), 2 matrix-core fragments (BF16),
                             3 slab factors (FP64/FP32) */
  int coarse_solver;      /* factorisation in use: TH_CSOLVE_LINES or TH_CSOLVE_ND */
  int coarse_levels;      /* ND: levels of the dissection tree (two launches each per solve) */
  int coarse_refine;      /* ND: iterative-refinement steps per coarse solve inside the FP64
                             preconditioner of th_solve (each one more solve with the factors
                             and a stencil residual): as many as bring the probe error to 1e-8 */
  double coarse_check;    /* max |A_c^{-1} (A_c x) - x| over the coarse vertices for the setup
                             probe x (unit-modulus entries) */
  int slab_packed;        /* slab factors: 1 when each symmetric G_t is stored once (the lower
                             block triangle as skewed 64 x 64 tiles plus a dense strip of its
                             last m mod 64 rows), 0 when stored whole; the environment variable
                             TH_SLAB_PACKED=0 or 1 at setup overrides the choice */
  int coarse_refine_exact;  /* ND: refinement steps of th_coarse_solve (FP64): as many as bring
                               the probe error to 1e-13, at most 3 */
  double coarse_check_pc;   /* the probe error at coarse_refine steps (coarse_check: at
                               coarse_refine_exact) */
} th_info;

/* Create a context on HIP device `hip_device`, ordering work on `hip_stream`
 * (a hipStream_t, NULL = default stream).  *out receives the context. */
th_status th_create(th_ctx **out, int hip_device, void *hip_stream);
void th_destroy(th_ctx *ctx);
const char *th_last_error(const th_ctx *ctx);
th_status th_get_info(const th_ctx *ctx, th_info *info);

/* Build the fine operator data and the smoother (Sec. 4.1, Alg. 2): per-cell
 * coefficients, the subdomains U^(i) and Omega^(i) = U^(i) + one cell layer,
 * and for every subdomain the data of its solve, computed on the device in
 * FP64 and stored in desc->gemm precision: the dense operator B_i =
 * diag(1/L_j) R_{U_i} (A_s^(i))^{-1} (n_U x n_Omega; for FP64/FP32 possibly
 * with the U x U block of the symmetric inverse kept once), or the slab
 * factors of A_s^(i) (th_layout; th_info.smoother_layout reports the choice).
 * Blocking.  Errors: TH_EINVAL (odd order, n < 1, k <= 0 or NaN, l_dd < 1, dim
 * not 2 or 3, a layout other than AUTO with BF16 storage), TH_EUNSUPPORTED (3-D
 * order above 4), TH_ENOMEM, TH_ENUMERIC (zero pivot). */
th_status th_setup_fine(th_ctx *ctx, const th_fine_desc *desc);

/* Build the coarse QSFEM quasi-FE matrix (Sec. 3.3, eq. element_wise_qsfem;
 * 27-point in 3-D) on the coarse vertex grid and factorise it once in FP64 on
 * the device (th_coarse_solver: nested dissection, or block elimination over
 * grid lines or planes; explicit inverses of the eliminated blocks).  Needs
 * th_setup_fine.  Blocking.  Errors: TH_EINVAL (also: surrogate network of the
 * other dimension's family, unknown solver), TH_ENOMEM, TH_ENUMERIC (a pivot
 * guard, or with TH_CSOLVE_ND a probe check above 1e-6). */
th_status th_setup_coarse(th_ctx *ctx, const th_coarse_desc *desc);

/* r = f - A u (fine Galerkin matrix, eq. bilin_form).  Stream-ordered. */
th_status th_residual(th_ctx *ctx, const void *u, const void *f, void *r,
                      int nrhs, th_dtype dt);

/* u <- CSDDSmoother(u, f) (Alg. 2): r = f - A u, n_dd DD steps on the
 * shifted operator with the averaged update (eq. RAS_like_update), u += v.
 * Stream-ordered. */
th_status th_smooth(th_ctx *ctx, void *u, const void *f, int nrhs, th_dtype dt);

/* rc = I_P^T r (adjoint of the Q_{p/2} interpolation, Sec. 4.2).  Stream-ordered. */
th_status th_restrict(th_ctx *ctx, const void *r, void *rc, int nrhs, th_dtype dt);

/* u += omega_c I_P uc (Sec. 4.2).  Stream-ordered. */
th_status th_prolong(th_ctx *ctx, const void *uc, void *u, double omega_c,
                     int nrhs, th_dtype dt);

/* uc = A_c^{-1} rc with the FP64 coarse factors (Alg. 1, coarse solve).
 * TH_C64 vectors are promoted to FP64 for the sweeps.  Stream-ordered. */
th_status th_coarse_solve(th_ctx *ctx, const void *rc, void *uc, int nrhs, th_dtype dt);

/* th_coarse_solve for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve, with every work vector (the nested-dissection update vectors, the
 * refinement residual and correction, the FP64 staging of TH_C64 vectors)
 * in a fixed 64 MiB device array per GPU that the library holds until the
 * process ends, instead of the context's buffers.  It allocates and frees
 * nothing.  Calls on one GPU share that array: calls that overlap in time on
 * one GPU (other streams, other contexts) race; nothing in it needs to start
 * at zero.  Results equal th_coarse_solve's.  Errors: those of
 * th_coarse_solve; TH_EINVAL when nrhs right-hand sides need more than 64 MiB
 * (nested dissection: nrhs x (update-vector length + 2 n_coarse) x 16 bytes,
 * plus 2 nrhs n_coarse x 16 bytes for TH_C64); TH_EUNSUPPORTED for the line
 * elimination of grids whose slabs it stages in context buffers (3-D).
 * Stream-ordered. */
th_status th_coarse_solve_noalloc(th_ctx *ctx, const void *rc, void *uc, int nrhs, th_dtype dt);

/* u <- TwoGridStep(u, f) (Alg. 1).  Stream-ordered. */
th_status th_twogrid(th_ctx *ctx, void *u, const void *f, int nrhs, th_dtype dt);

/* Solve A u = f (eq. bilin_form, Sec. 2-3.1) for nrhs right-hand sides
 * (TH_C128 device vectors, u overwritten, x0 = 0) with the two-grid
 * preconditioner f -> TwoGridStep(0, f) of Sec. 4 (Alg. 1: n_s smoothing steps
 * of Alg. 2, coarse-grid correction with omega_c, n_s smoothing steps) inside
 * the outer iteration of opts->krylov: GMRES in FP64 (matvec, residual,
 * orthogonalisation, Hessenberg) or the stationary iteration.  Blocking.
 * Returns TH_OK only when every RHS meets opts->rtol on its true FP64
 * residual; TH_ENOTCONV when maxit is reached first (u holds the last
 * iterate, stats filled, stats->rel_res > rtol); TH_EINVAL (rtol <= 0,
 * maxit < 1, unknown method or dtype, nrhs > max_rhs); TH_ESTATE (no coarse
 * setup); TH_ENOMEM (Krylov basis); TH_ENUMERIC (NaN/Inf in f, the Arnoldi
 * process or the residual). */
th_status th_solve(th_ctx *ctx, const void *f, void *u, int nrhs,
                   const th_solve_opts *opts, th_solve_stats *stats);

/* Kernel timing for measurement.  While enabled, HIP events are recorded on
 * the context stream around every launch of the library's kernels, grouped by
 * the kernel classes below.  th_timing_enable(ctx, 1) clears the totals;
 * th_timing_get synchronises the stream and returns, for one class, the summed
 * GPU time in milliseconds and the number of launches since then. */
typedef enum {
  TH_KT_DD_APPLY = 0,   /* batched subdomain solves Y_i = B_i X_i */
  TH_KT_DD_ACCUM = 1,   /* averaged update of the smoother */
  TH_KT_OPERATOR = 2,   /* matrix-free fine operator (residual / matvec) */
  TH_KT_RESTRICT = 3,
  TH_KT_PROLONG = 4,
  TH_KT_COARSE = 5,     /* coarse forward/backward sweeps */
  TH_KT_KRYLOV = 6,     /* GMRES vector kernels */
  TH_KT_COUNT = 7
} th_kernel_class;

th_status th_timing_enable(th_ctx *ctx, int enable);
th_status th_timing_get(th_ctx *ctx, int kernel_class, double *total_ms, long long *launches);

/* ------------------------------------------------------------------------
 * Dispersion-matched coarse stencils (a project addition motivated by the
 * footnote of Sec. 1: the coarse level should match the fine, not the true,
 * dispersion relation).  A sample is (eta_c, p, shift): eta_c = h_c k of a
 * coarse cell (h_c = 2h/p), the order p, and shift = eps / k^2.
 *
 * Plain fit: e_m = r(t_m) / kh - 1, the relative error of the fine Q_p
 * discrete wavenumber (Sec. 6.2) along t_1 = pi/16 and t_2 = 3 pi/16, and the
 * 9-point weights (q0, q_edge, q_diag) of the QSFEM family (Sec. 3.2) whose
 * zero set passes through those fine wave vectors, scaled so that the symbol
 * at 0 is -eta^2.  Valid for kh = eta_c p / 2 < pi.  Host computation.
 *   samples: HOST n x 3; e_out: HOST n x 2 or NULL; q_out: HOST n x 3 or NULL. */
th_status th_plain_fit(const double *samples, int n, double *e_out, double *q_out);

/* 3-D analogue (project definition; the paper treats 2-D): the compact
 * 27-point family with classes centre P0 = 8, face P1, edge P2, corner P3,
 *   sigma(xi) = P0 + 2 P1 sum c_i + 4 P2 sum_{i<j} c_i c_j + 8 P3 c_1 c_2 c_3,
 * c_i = cos(h_c xi_i), whose zero set passes through the fine Q_p discrete
 * wave vectors along the normalised directions (1, .2, .1), (1, .6, .3),
 * (1, .9, .7), scaled so that sigma(0) = -eta^2; quasi-FE weights
 * (q0, q_face, q_edge, q_corner) = N (P0 / 8, P1 / 4, P2 / 2, P3).
 *   samples: HOST n x 3; e_out: HOST n x 3 or NULL; q_out: HOST n x 4 or NULL. */
th_status th_plain_fit3d(const double *samples, int n, double *e_out, double *q_out);

/* Surrogate network 3 -> 64 -> 64 -> n_out (SiLU), inputs standardised
 * samples, outputs standardised log(max(-e_m, 0) + 1e-13) of the fine
 * dispersion errors of a stencil family: n_out = 2 for the 9-point family
 * (th_plain_fit's e_m, 2-D problems), 3 for the 27-point family
 * (th_plain_fit3d's e_m, 3-D problems).  FP32 master weights with a BF16
 * copy, FP32 accumulation.  Weight layout (n_params = 4355 + 65 n_out floats:
 * 4546 or 4611): W1 (64 x 3 row-major), b1 (64), W2 (64 x 64), b2 (64),
 * W3 (n_out x 64), b3 (n_out).  Below, arrays of "n_out" values follow the
 * network's family. */
typedef struct {
  int epochs;           /* passes over the samples */
  int batch;            /* samples per step (multiple of 64) */
  double lr;            /* Adam learning rate */
  int bf16;             /* 1: forward/backward with the BF16 weight copy */
} th_mlp_train_opts;

typedef struct {
  double loss_first, loss_last;  /* mean squared error of the first / last step */
  int steps;
  double t_targets_s, t_train_s;  /* plain-fit targets on the host / training on the device */
} th_mlp_train_stats;

th_status th_mlp_create(th_mlp **out, int hip_device, void *hip_stream);  /* 2-D family */
/* dim 2: the 9-point family, dim 3: the 27-point family; TH_EINVAL otherwise */
th_status th_mlp_create_family(th_mlp **out, int hip_device, void *hip_stream, int dim);
/* the network's dimension and parameter count */
th_status th_mlp_info(const th_mlp *m, int *dim, int *n_params);
void th_mlp_destroy(th_mlp *m);
const char *th_mlp_last_error(const th_mlp *m);
th_status th_mlp_num_params(int *n_params);  /* of the 2-D family */
/* theta: HOST FP32 weights in the layout above (the BF16 copy is refreshed) */
th_status th_mlp_set_weights(th_mlp *m, const float *theta, int n_params);
th_status th_mlp_get_weights(const th_mlp *m, float *theta, int n_params);
/* standardisation: x_std = (x - in_mean) / in_std, y_std = (y - out_mean) / out_std */
th_status th_mlp_set_scaling(th_mlp *m, const double *in_mean, const double *in_std,
                             const double *out_mean, const double *out_std);
th_status th_mlp_get_scaling(const th_mlp *m, double *in_mean, double *in_std, double *out_mean,
                             double *out_std);
/* Loss (mean squared error) and gradient for HOST standardised data
 * x_std (n x 3) and y_std (n x n_out), computed by the device kernels; bf16 selects
 * the BF16 weight copy.  grad: HOST n_params floats. */
th_status th_mlp_loss_grad(th_mlp *m, const float *x_std, const float *y_std, int n, int bf16,
                           double *loss, float *grad);
/* Train on n HOST samples: plain-fit targets on the host, standardisation
 * from the samples, Adam steps on the device from the current weights. */
th_status th_mlp_train(th_mlp *m, const double *samples, int n, const th_mlp_train_opts *opts,
                       th_mlp_train_stats *stats);
/* Device inference for n HOST samples: e_out (HOST n x n_out) = predicted e_m. */
th_status th_mlp_predict(th_mlp *m, const double *samples, int n, int bf16, double *e_out);
/* Coarse stencils from the network for n HOST samples of one order p, all on
 * the device: inference (BF16 weights), weights q_out (HOST n x 3 for the
 * 9-point family, n x 4 for the 27-point family) from the predicted e_m by
 * the plain-fit formulas, and mismatch_out (HOST n): the largest distance,
 * relative to eta, between the stencil's zero set and the fine Q_p
 * dispersion curve over the symmetry sector of wave directions (the curve
 * traced through the separation mu(theta_x) + mu(theta_y) [+ mu(theta_z)] =
 * (kh)^2 of the tensor-product symbol at 16 points in 2-D, 21 in 3-D; one
 * Newton step of the coarse symbol along each point's ray).  Infinite where
 * the curve leaves the acoustic branch.  TH_COARSE_MLP sends a cell back to
 * the plain fit when its mismatch exceeds fallback_tau.  Errors: TH_EINVAL
 * (samples of several orders), TH_ESTATE (no weights). */
th_status th_mlp_stencils(th_mlp *m, const double *samples, int n, double *q_out,
                          double *mismatch_out);

#ifdef __cplusplus
}
#endif
#endif /* TH_H */
