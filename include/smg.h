/* smg.h -- C ABI of the MI355X collective multigrid library (libsmg.so).
 *
 * Solves the block saddle-point system S x = f of a linear-quadratic optimal
 * control problem under uncertainty (Ciaramella, Nobile, Vanzan, arXiv
 * 2302.13680, eq. (2) and eq. full_space_optimality_system):
 *
 *     [ C_1            A_1^T          ] [ y_1 ]   [ f_Y,1 ]
 *     [     ...             ...       ] [ ... ]   [  ...  ]
 *     [         C_N             A_N^T ] [ y_N ]   [ f_Y,N ]
 *     [             G   D_1 ...  D_N  ] [  u  ] = [  f_U  ]
 *     [ A_1         E_1               ] [ p_1 ]   [ f_P,1 ]
 *     [     ...     ...               ] [ ... ]   [  ...  ]
 *     [         A_N E_N               ] [ p_N ]   [ f_P,N ]
 *
 * on an n x n interior grid of the unit square (homogeneous Dirichlet), with
 *   - A_j the symmetric 5-point stencil built from face coefficients
 *     (finite differences scaled by h^2; A_j^T = A_j): for node (x, k)
 *       (A_j v)(x,k) = (kW+kE+kS+kN) v(x,k) - kW v(x-1,k) - kE v(x+1,k)
 *                                           - kS v(x,k-1) - kN v(x,k+1),
 *     kW = kx(k, x), kE = kx(k, x+1), kS = ky(k, x), kN = ky(k+1, x);
 *   - C_j = c_j I, D_j = d_j I, E_j = e_j I, G = g I (diagonal blocks with one
 *     value per sample, e.g. c_j = zeta_j h^2, d_j = e_j = -h^2, g = nu h^2).
 *
 * The solver is the collective multigrid V-cycle (Alg. 1) with the
 * red-black collective Gauss-Seidel smoother whose node solve is
 * eq. solution_reduced_system, used stationary, as the right preconditioner
 * of GMRES(m), or in FP32 inside FP64 iterative refinement.
 *
 * LAYOUTS (all device memory; samples innermost):
 *   vector x or f, length (2N+1) n^2 elements:
 *       [ Y block: [n][n][N] | U block: [n][n] | P block: [n][n][N] ]
 *       i.e. Y(j, x, k) at  (k*n + x)*N + j,  U(x, k) at N*n*n + k*n + x,
 *            P(j, x, k) at  (N+1)*n*n + (k*n + x)*N + j.
 *   kx: [n][n+1][N]  kx(k, f, j) = coefficient of sample j on the x-face
 *       between columns f-1 and f of row k (f = 0 and f = n touch the boundary)
 *   ky: [n+1][n][N]  ky(g, x, j) = coefficient on the y-face between rows
 *       g-1 and g of column x.
 *   This is eq. (2)'s ordering with every block transposed to node-major,
 *   sample-minor order, so that one wavefront holds the samples of a node.
 *
 * OWNERSHIP: all device buffers (blocks, x, f, workspace) belong to the
 * caller and must outlive the context; the library never frees them.  The
 * finest-level kx/ky are referenced, not copied.  The context struct itself
 * is allocated by smg_setup and freed by smg_destroy.  Work is enqueued on the
 * caller's HIP stream; calls that report iteration counts or norms
 * synchronize that stream.  A context is not thread-safe: one context per
 * stream.
 *
 * ERRORS: every int-returning call returns SMG_OK (0), SMG_NOT_CONVERGED (1,
 * stats are filled) or a negative code; smg_strerror maps codes to text and
 * smg_last_error(ctx) gives detail.  Arguments are validated on the host
 * before any launch.
 */
#ifndef SMG_H
#define SMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SMG_OK 0
#define SMG_NOT_CONVERGED 1
#define SMG_EINVAL (-1)       /* bad size, pointer or option */
#define SMG_ESINGULAR (-2)    /* non-positive diagonal or node denominator, singular coarsest block */
#define SMG_EHIP (-3)         /* a HIP runtime call failed */
#define SMG_ENONFINITE (-4)   /* a residual norm became NaN or Inf */
#define SMG_EWORKSPACE (-5)   /* workspace missing or too small */

/* arithmetic of the V-cycle */
#define SMG_F64 0             /* everything in FP64 */
#define SMG_F32 1             /* smoother, residual and transfers in FP32, coarsest solve,
                                 outer residual and Krylov updates in FP64 */

/* solver choice for smg_solve */
#define SMG_VCYCLE 0          /* stationary V-cycles (FP32 mode: FP64 refinement, one FP32 cycle per step) */
#define SMG_GMRES 1           /* right-preconditioned GMRES(m) (FP32 mode: FP64 refinement
                                 around flexible GMRES(m) with the FP32 cycle) */

typedef struct smg_ctx smg_ctx;

typedef struct {
  int n;              /* interior nodes per direction: (coarsest_n+1) 2^k - 1 */
  int nsamples;       /* N >= 1 (at most 2048; the batched solver takes at most 512) */
  int coarsest_n;     /* odd, 1..7; grid of the direct solve (0 selects 7) */
  int pre, post;      /* smoothing sweeps n1, n2 per level (red + black half-sweeps each) */
  double theta;       /* relaxation of the node update (1 = Gauss-Seidel; 0 selects 1) */
  int precision;      /* SMG_F64 or SMG_F32 */
  int gmres_restart;  /* basis size m reserved for GMRES (0 = no Krylov storage) */
  int flags;          /* SMG_FLAG_* bits */
  int strip;          /* smoother traversal: vertical strips of this many columns (even), each
                         visited row by row, so that values shared by neighbouring rows are
                         reused from L2; 0 or >= n = row-major order.  Any value gives the
                         same iterates (a half-sweep updates one colour from the other). */
  int sweep_rows;     /* rows per segment of the one-launch red+black sweep (see
                         SMG_FLAG_HALFSWEEPS); 0 = as many segments as keep every wave of the
                         launch resident at once.  A value > 0 also enables that sweep on
                         levels below its size threshold.  Any value gives the same iterates. */
} smg_desc;

/* flags */
#define SMG_FLAG_EAGER 1      /* launch every V-cycle kernel by kernel instead of replaying a
                                 captured hipGraph (the default captures one graph per distinct
                                 (x, f) buffer pair on first use and replays it afterwards) */
#define SMG_FLAG_UNFUSED 2    /* separate residual, restriction, prolongation and zero-fill
                                 kernels (the default fuses them into neighbouring kernels when
                                 theta = 1; both compute the same iteration) */
#define SMG_FLAG_JACOBI 4     /* smooth with damped collective Jacobi steps (eq.
                                 collective_smoothing; the smoother of the paper's experiments,
                                 which use theta = 0.5) instead of red-black collective
                                 Gauss-Seidel sweeps; theta is the damping and pre / post count
                                 Jacobi steps.  Not accepted by the batched solver. */
#define SMG_FLAG_SSN 8        /* reserve the semismooth Newton solver's buffers in the workspace
                                 (two vectors and six node-sized arrays) */
#define SMG_FLAG_CVAR 16      /* reserve the risk-averse solver's buffers (eight vectors, the
                                 rank-one vectors z_j and per-sample arrays); FP64 contexts only */
#define SMG_FLAG_HALFSWEEPS 32 /* smooth with one launch per colour on every level.  By default,
                                 on levels whose two half-sweeps move at least 512 MB with
                                 65..256 samples (two to four per lane), and on every level with 33..256
                                 samples (64 lanes per node; FP32 pairs: 65..256) when sweep_rows
                                 is set, with theta = 1, no node factors and no domain, a whole
                                 red+black sweep is one launch out of place between the level
                                 iterate and a second buffer, reading every face coefficient
                                 once, the coarse correction ahead of post-smoothing is a pass
                                 over the black nodes only, the residual after two or more
                                 pre-smoothing sweeps is restricted from the black nodes' change
                                 in the last one (see smg_residual_restrict_after_sweep), every
                                 sweep but the last post-smoothing one stores the black nodes'
                                 y and p only (no later step reads the rest), and the finest
                                 residual and operator application run in column walks; both
                                 compute the same iteration (the same arithmetic per node, up to
                                 the order of the restriction's sums and the rounding of the
                                 node solves in the restricted residual) */

typedef struct {
  const double *kx;   /* device, [n][n+1][N] */
  const double *ky;   /* device, [n+1][n][N] */
  const double *c;    /* host, [N]: C_j = c_j I (> 0) */
  const double *d;    /* host, [N]: D_j = d_j I */
  const double *e;    /* host, [N]: E_j = e_j I */
  double g;           /* G = g I (> 0) */
  const double *ctrl; /* host, [n][n] or NULL: control mask m_i in [0, 1] (local control, e.g.
                         the indicator of the control region): the node entries of D_j and E_j
                         become m_i d_j and m_i e_j, so where m_i = 0 the node solve has no
                         control (eq. solution_reduced_system2) and, with f_U = 0 there,
                         u_i = 0.  Coarse levels take the mask by injection.  NULL: the
                         control acts everywhere.  Values outside [0, 1]: SMG_EINVAL. */
  const double *domain; /* host, [n][n] or NULL: 1 inside the domain, 0 outside (e.g. the
                         paper's L-shape (0,1)^2 minus [1/2,1)^2: the nodes with x, y >= 1/2
                         removed).  Nodes outside are homogeneous Dirichlet nodes: their
                         rows of S are zero, every kernel keeps x there at zero and reads
                         those zeros as the Dirichlet values of the nodes inside, and the
                         solvers (smg_vcycle, smg_gmres_precond, smg_solve, smg_ssn_solve)
                         zero x there on entry; the step entry points expect x zero there.
                         Coarse levels by injection: the domain's edges must lie on grid
                         lines of every level (true for the L-shape).  Values other than 0
                         and 1: SMG_EINVAL.  Not accepted by the batched solver.  NULL:
                         the whole square. */
  double control_growth; /* factor by which d_j, e_j and g grow per coarsening (0: 4, the
                         h^2 of an area mass, like c_j).  2 for a control on a line (the
                         boundary control by reflection: the 1D mass h of the control
                         line).  Other values: SMG_EINVAL unless in (0, 16]. */
} smg_blocks;

typedef struct {
  int iterations;       /* V-cycles (stationary), GMRES iterations, or refinement steps */
  int inner_iterations; /* preconditioner applications (V-cycles) in total */
  int restarts;         /* GMRES restarts */
  double relres;        /* final ||f - S x||_2 / ||f||_2 in FP64 */
  double relres_y, relres_u, relres_p; /* per block row, each relative to ||f||_2 */
  double time_ms;       /* wall time of the call, host clock */
  double *history;      /* optional caller buffer: relative residual per iteration */
  int history_cap;      /* its length (0 = none) */
  int history_len;      /* entries written */
} smg_stats;

/* Parameters of the semismooth Newton solver (Section 5, eq. l1_OCP and Algorithm 2). */
typedef struct {
  double nu;          /* nu > 0, the control cost */
  double beta;        /* beta >= 0, the L^1 weight */
  double a, b;        /* box a < 0 < b on the control (-INFINITY / INFINITY: no bound) */
  double mass;        /* M = mass I, the lumped mass matrix (h^2 for these grids) */
  double tol;         /* stop once phi(u) = sqrt(F^T M F) <= tol (the paper: 1e-9) */
  double inner_rtol;  /* relative residual of every linear solve (the paper: 1e-11) */
  int inner_method;   /* SMG_VCYCLE or SMG_GMRES (V-cycle-preconditioned) */
  int maxit;          /* Newton iterations at most */
  int inner_maxit;    /* iterations of each linear solve at most */
  double sigma, rho;  /* line search: sufficient decrease sigma, step factor rho (0: 1e-4, 1/2) */
} smg_ssn_params;

typedef struct {
  int iterations;       /* Newton iterations */
  int inner_total;      /* linear-solver iterations over all Newton systems */
  int init_iterations;  /* iterations of the initial state and adjoint solve */
  double phi_final;     /* final merit phi(u) */
  double time_ms;       /* wall time of the call, host clock */
  double *phi;          /* optional caller buffers of cap entries: merit per iterate (u^0, u^1, ...), */
  double *gamma;        /*   step length and linear-solver iterations per Newton iteration */
  int *inner;
  int cap;
  int len;              /* iterates recorded (iterations + 1) */
} smg_ssn_stats;

/* Bytes of device workspace smg_setup needs for this descriptor.  Pure host
 * computation; returns 0 for an invalid descriptor. */
size_t smg_workspace_bytes(const smg_desc *desc);

/* Build the level hierarchy (Section 3: nested grids n -> (n-1)/2 with coarse
 * operators by rediscretization: face coefficients averaged pairwise, the
 * diagonal blocks scaled by 4 per level), check a > 0 and the node
 * denominators of eq. solution_reduced_system (c, d e with the sign that makes
 * G + sum_j d_j c_j e_j / a_j^2 > 0), and factor the coarsest level (its A_j
 * and the control Schur complement inverted in FP64).  workspace: device
 * buffer of at least smg_workspace_bytes(desc) bytes, 256-byte aligned.
 * stream: hipStream_t (NULL = default stream).  On success *out is a new
 * context. */
int smg_setup(const smg_desc *desc, const smg_blocks *blocks, void *workspace,
              size_t workspace_bytes, void *stream, smg_ctx **out);

void smg_destroy(smg_ctx *ctx);

const char *smg_strerror(int code);
const char *smg_last_error(const smg_ctx *ctx);

int smg_num_levels(const smg_ctx *ctx);
int smg_level_n(const smg_ctx *ctx, int level);

/* Sx = S x on the finest level, FP64 (eq. (2)).  x and Sx: device vectors. */
int smg_apply(smg_ctx *ctx, const double *x, double *Sx);

/* r = f - S x on the finest level, FP64; if norms != NULL it receives (host)
 * { ||r||, ||r_Y||, ||r_U||, ||r_P|| } (2-norms). */
int smg_residual(smg_ctx *ctx, const double *x, const double *f, double *r, double *norms);

/* The same residual r = f - S x for callers that cannot allocate device memory
 * or read back to the host (code under HIP graph capture, serving loops): the
 * kernels' per-block partial sums live in a static device array of the library
 * (8.4 MB per GPU, held until the process ends; enough for 1023 x 1023 grids)
 * instead of the context's workspace, and the five norms
 * { ||r||, ||r_Y||, ||r_U||, ||r_P||, ||f|| } go to norms_dev (device, 5
 * doubles) with no host synchronization.  Launches kernels only (no
 * allocation, no memset, no copy).  Calls that overlap on one GPU (other
 * streams or threads) share that array and race.  SMG_EWORKSPACE when the grid
 * needs more scratch than the array holds, SMG_EINVAL with rank-one terms set
 * (smg_set_lowrank) or null pointers. */
int smg_residual_static(smg_ctx *ctx, const double *x, const double *f, double *r, double *norms_dev);

/* One half-sweep of the collective Gauss-Seidel smoother on level `level`
 * (eq. collective_smoothing, node solve eq. solution_reduced_system): every
 * node with (x + k) % 2 == colour gets (1-theta) x_i + theta S~_i^{-1} b_i.
 * x, f: FP64 device vectors of that level's size. */
int smg_smooth(smg_ctx *ctx, int level, int colour, double *x, const double *f);

/* One whole sweep (red then black half-sweep, Section 3 with collective
 * Gauss-Seidel) on level `level` from xin into xout (FP64 device vectors of the
 * level's size that must not overlap; f likewise); xout equals xin after
 * smg_smooth with colour 0 and then 1 (theta = 1 required).  Where the
 * one-launch sweep applies (see SMG_FLAG_HALFSWEEPS) it is that single launch;
 * otherwise xin is copied to xout and the two half-sweeps run there.  *one
 * (may be NULL) tells which.  SMG_EINVAL for theta != 1 or aliasing vectors. */
int smg_sweep(smg_ctx *ctx, int level, const double *xin, double *xout, const double *f, int *one);
/* The same in FP32 arithmetic on FP32 vectors (SMG_F32 contexts). */
int smg_sweep32(smg_ctx *ctx, int level, const float *xin, float *xout, const float *f, int *one);

/* Device-to-device copy of `bytes` (a multiple of 16, both pointers 16-byte
 * aligned) by a plain streaming kernel (16-byte non-temporal accesses, four in
 * flight per lane), on `stream` (hipStream_t, NULL = default): the
 * achievable-bandwidth reference quoted next to the kernels' rooflines.
 * SMG_EINVAL for bad sizes or alignment. */
int smg_stream_copy(void *dst, const void *src, size_t bytes, void *stream);

/* The same half-sweep in FP32 arithmetic on FP32 device vectors x, f of the
 * level's size, with the context's FP32 copy of the level operator (the
 * smoother of the FP32 cycle).  SMG_EINVAL unless the context was set up with
 * precision SMG_F32. */
int smg_smooth32(smg_ctx *ctx, int level, int colour, float *x, const float *f);

/* coarse = R fine (R = P^T, full weighting with weights 1, 1/2, 1/4), fine of
 * level `level`, coarse of level + 1, all 2N+1 fields.  FP64 device vectors. */
int smg_restrict(smg_ctx *ctx, int level, const double *fine, double *coarse);

/* One damped collective Jacobi step on level `level` (eq. collective_smoothing):
 * xout = x + theta D^{-1} (f - S x), D the block diagonal of the (2N+1)x(2N+1)
 * node blocks of eq. reduced_matrices, theta the context's.  x, xout, f: FP64
 * device vectors of that level's size; xout must not alias x (SMG_EINVAL). */
int smg_jacobi(smg_ctx *ctx, int level, const double *x, double *xout, const double *f);

/* coarse = R (f - S x) in one pass: the residual of Alg. 1 on level `level`
 * restricted to level + 1 without storing the fine residual (the result of
 * smg_residual followed by smg_restrict up to rounding order, except that the U
 * block is restricted within the control space: U residuals of fine nodes without
 * a control (factors of D_j and E_j both zero) are dropped, and a coarse node
 * whose coincident fine node has none gets a zero U row).  x, f: FP64 device vectors
 * of level `level` (f is that level's right-hand side); coarse: level + 1.
 * SMG_EINVAL if `level` has no coarser level. */
int smg_residual_restrict(smg_ctx *ctx, int level, const double *x, const double *f, double *coarse);

/* The same restriction right after a sweep (Alg. 1's residual following the
 * pre-smoothing, Section 3 with collective Gauss-Seidel): xnew must be one
 * smg_sweep of xold with right-hand side f (theta = 1); xold, xnew, f: FP64
 * device vectors of level `level` (xold and xnew distinct), coarse: level + 1.
 * Each node solve makes its own block row exact for the values it read, so the
 * black rows and every U row of f - S xnew vanish and a red row is the coupling
 * through its four faces to the blacks' change xnew - xold; where the column
 * walk applies (the one-launch sweep's levels, see SMG_FLAG_HALFSWEEPS) coarse
 * is formed from that change without reading f and *from_change (may be NULL)
 * is set to 1; otherwise it is smg_residual_restrict(xnew, f) and 0.  Equal to
 * R (f - S xnew) up to the rounding of the node solves.  SMG_EINVAL as
 * smg_residual_restrict, or for xold == xnew. */
int smg_residual_restrict_after_sweep(smg_ctx *ctx, int level, const double *xold, const double *xnew,
                                      const double *f, double *coarse, int *from_change);

/* fine += P coarse (bilinear interpolation; Alg. 1 coarse correction).  The U
 * block is prolongated into the control space only: fine nodes whose factors
 * of D_j and E_j are both zero (no control there, e.g. outside a local control
 * region or off a boundary-control line) keep their u. */
int smg_prolong_add(smg_ctx *ctx, int level, const double *coarse, double *fine);

/* X = S^{-1} F on the coarsest level (Alg. 1 direct solver), FP64. */
int smg_coarse_solve(smg_ctx *ctx, const double *F, double *X);

/* Copy the face coefficients the hierarchy holds for `level` into device
 * buffers kx [n_l][n_l+1][N] and ky [n_l+1][n_l][N] (FP64). */
int smg_level_faces(smg_ctx *ctx, int level, double *kx, double *ky);

/* ncycles V-cycles (Alg. 1) in place on the finest level: x <- Vcycle(x, f).
 * In SMG_F32 mode x and f are rounded to FP32 on entry and x is widened on
 * exit. */
int smg_vcycle(smg_ctx *ctx, double *x, const double *f, int ncycles);

/* GMRES(restart) preconditioned on the right by one V-cycle from a zero guess,
 * on the initial guess in x (Section 3.2 experiments; the monitored residual
 * is the unpreconditioned one).  Stops when ||f - S x|| <= rtol ||f|| or after
 * maxit iterations.  restart <= desc.gmres_restart.  In SMG_F32 mode the
 * basis stays FP64 and the preconditioner is the FP32 cycle (flexible GMRES). */
int smg_gmres_precond(smg_ctx *ctx, double *x, const double *f, int restart, double rtol,
                      int maxit, smg_stats *stats);

/* Solve S x = f to ||f - S x||_2 <= rtol ||f||_2 starting from the x given.
 * method SMG_VCYCLE or SMG_GMRES (see above); in SMG_F32 mode both run as FP64
 * iterative refinement around the FP32 cycle (maxit bounds the refinement
 * steps; each GMRES-based step stops at inner_rtol = 1e-5 relative to the
 * current residual). */
int smg_solve(smg_ctx *ctx, double *x, const double *f, int method, double rtol, int maxit,
              smg_stats *stats);

/* how node factors reach coarse levels (smg_set_node_factors) */
#define SMG_COARSEN_INJECT 0  /* coarse node (X, K) takes fine node (2X+1, 2K+1) */
#define SMG_COARSEN_FULL 1    /* full-weighting average of the 3 x 3 fine nodes around it, weights
                                 (1/4)(1/2)^(|dx|+|dk|): the row-lumped diagonal of R diag(v) P */

/* Node factors of D_j and E_j: the node entries become md_i d_j and me_i e_j
 * on every level (coarse levels level by level by `coarsening`, one of
 * SMG_COARSEN_*), and the per-node denominators and the coarsest Schur
 * complement are rebuilt.  Local control is md = me = the control mask
 * (smg_setup's ctrl, by injection); the Newton system of Section 5
 * (eq. full_space_optimality_systeMemismooth2) is md = the active-set
 * indicator, me = 1, by full weighting (the V-cycle then needs a third to a
 * fifth of the cycles injection needs).  md, me: device, [n][n] (row k,
 * column x) of the finest level, values in [0, 1]; NULL: 1 everywhere.
 * Replaces the control mask given to smg_setup.  Synchronizes the context's
 * stream.  A value outside [0, 1] or not finite, or an unknown coarsening:
 * SMG_EINVAL, nothing changed. */
int smg_set_node_factors(smg_ctx *ctx, const double *md, const double *me, int coarsening);

/* ------------------------------------------------------- semismooth Newton
 * The control problem with an L^1 penalty and box constraints (Section 5,
 * eq. l1_OCP), solved by the globalized semismooth Newton method of
 * Algorithm 2 with the collective multigrid for every Newton system.
 *
 * The context must have SMG_FLAG_SSN and hold the Newton
 * system's blocks (eq. full_space_optimality_systeMemismooth2 with the
 * adjoint rescaled by the sample weights, p~_j = zeta_j p_j): C_j = zeta_j M,
 * E_j = -M and faces as in the linear-quadratic problem, and the U row as
 * printed, G = M and D_j = -M / nu.  E[p] = sum_j zeta_j p_j is then the sum
 * of the P block's samples at a node.  Vectors in the node layout, FP64; in
 * SMG_F32 mode every linear solve is FP64 refinement around FP32 cycles (see
 * smg_solve), which reaches the same FP64 tolerances. */

/* Per node of x (device, finest level): w = E[p] (device [n][n]); when F and
 * chi are given (both or neither) also F(u) of the discrete optimality
 * condition, the indicator chi of the active sets I+ u I- (eq. activesets,
 * 1.0 or 0.0) and, if phi is given, the merit phi = sqrt(F^T M F) (host). */
int smg_ssn_eval(smg_ctx *ctx, const double *x, const smg_ssn_params *prm, double *w, double *F,
                 double *chi, double *phi);

/* Line-search merits: phis[q] = phi(u + gammas[q] du) with the trial E[p]
 * taken as w + gammas[q] dw (exact: y and p are affine in u), q < ng <= 8.
 * u, du, w, dw: device [n][n]; gammas, phis: host. */
int smg_ssn_merit(smg_ctx *ctx, const double *u, const double *du, const double *w, const double *dw,
                  const smg_ssn_params *prm, int ng, const double *gammas, double *phis);

/* Algorithm 2.  x (device, node layout): on entry its U block is u^0 and its
 * Y and P blocks are the initial guess of the first solve (zero is fine); on
 * exit (y, u, p~) of the last iterate.  f: the linear-quadratic right-hand
 * side (f_Y,j = zeta_j M y_d, f_P,j = M f; its U block is not used).  Steps:
 * the state and adjoint equations for u^0 (the system with D_j = 0 and U
 * block M u^0); then until phi(u^k) <= tol: node factors md = chi(u^k),
 * me = 1, the Newton system with right-hand side (0, -M F(u^k), 0) solved from
 * zero to inner_rtol (coarse levels take the active set by full weighting), the first step length of 1, rho, rho^2, ... (at most 64)
 * with phi(u + gamma du) - phi(u) <= -sigma phi(u), x += gamma dx.  The
 * context keeps the last node factors.  Returns SMG_OK, SMG_NOT_CONVERGED
 * (maxit reached, no step of sufficient decrease, or the initial solve did not
 * converge) or an error. */
int smg_ssn_solve(smg_ctx *ctx, double *x, const double *f, const smg_ssn_params *prm,
                  smg_ssn_stats *stats);

/* ------------------------------------------------------- risk-averse (CVaR)
 * The smoothed-CVaR control problem (Section 6, eq. OCP) and the nonlinear
 * preconditioned Newton method of Algorithm 3.  Its Newton matrices J_11 are
 * the linear-quadratic operator with per-sample C_j = c_j I plus one rank-one
 * term w_j z_j z_j^T per sample in the Y-Y blocks (eq. equation_C). */

/* Per-sample state-mass values of the finest level: C_j = c[j] I (host, N
 * values, each >= 0 and finite), coarse levels 4^l c_j; the per-node control
 * denominators and the coarsest factorization are rebuilt.  SMG_EINVAL for a
 * bad value. */
int smg_set_sample_weights(smg_ctx *ctx, const double *c);

/* Rank-one terms of the finest level: the Y-Y block of sample j becomes
 * C_j + w_j z_j z_j^T.  z: device [n][n][N] (the Y block's layout), w: device
 * [N]; both copied.  From then on smg_apply, smg_residual, smg_gmres_precond
 * and smg_solve(SMG_GMRES) use that operator, with the V-cycle of the operator
 * without them as the preconditioner; smg_solve(SMG_VCYCLE) and the cycle and
 * step entry points keep the operator without them.  z = w = NULL clears.
 * Needs SMG_FLAG_CVAR (else SMG_EINVAL). */
int smg_set_lowrank(smg_ctx *ctx, const double *z, const double *w);

typedef struct {
  double lambda;      /* confidence level, 0 <= lambda < 1 */
  double eps;         /* smoothing width of g_eps (eq. smoothapproximation), > 0 */
  double mass;        /* M = mass I, the lumped mass (h^2 for these grids) */
  const double *zeta; /* host [N]: sample weights (sum 1) */
  double tol;         /* outer stop |F(t)| <= tol (the paper: 1e-6) */
  double inner_tol;   /* h(t): stop once max(||F_1|| / ||F_1(x^0)||, ||F_1||) <= inner_tol (the
                         paper: 1e-8; x^0 the start of that Newton iteration) */
  double lin_rtol;    /* GMRES relative residual of every Newton system (1e-9) */
  int maxit;          /* outer iterations at most */
  int inner_maxit;    /* Newton iterations per evaluation of h(t) at most */
  int lin_maxit;      /* GMRES iterations per system at most (the paper: 80) */
  double sigma, rho;  /* line search on t (0: 1e-4, 1/2) */
  int inner_rule;     /* 0: the printed rule with max (both parts small); SMG_CVAR_INNER_MIN:
                         min (either part small), a named option that is not the paper's */
  int inner_full_steps; /* 0: each Newton step for h(t) halved (at most 30 times) until
                         ||F_1(x + a dx)|| <= (1 - 1e-4 a) ||F_1(x)|| (the paper names Newton's
                         method without its globalization; full steps cycle on its
                         Monte Carlo problems); the iteration ends without the step when no
                         halving decreases ||F_1|| <= inner_tol (the rounding floor), takes
                         the last halving otherwise; 1: full Newton steps */
} smg_cvar_params;

#define SMG_CVAR_INNER_MAX 0
#define SMG_CVAR_INNER_MIN 1

typedef struct {
  int outer;            /* outer (preconditioned) Newton iterations */
  int inner_total;      /* Newton iterations for h(t) over the whole run */
  int linear_solves;    /* GMRES solves (Newton systems and the J_11 solves of F'(t)) */
  int linear_total;     /* GMRES iterations over all of them */
  double t;             /* final t */
  double F_final;       /* |F(t)| at the final iterate */
  double time_ms;
  double *F;            /* optional caller buffer of cap entries: |F(t^k)| per iterate */
  int cap;
  int len;
  int inner_capped;     /* evaluations of h(t) that ended at inner_maxit (with the printed rule:
                           a warm start within 1/inner_tol of the rounding floor) */
  int inner_stalled;    /* evaluations that ended because no halving decreased ||F_1|| with
                           ||F_1|| <= inner_tol (the rounding floor) */
  int *inner_counts;    /* optional caller buffer of inner_cap entries: Newton count of every
                           evaluation of h(t), in order */
  int inner_cap;
  int inner_len;
} smg_cvar_stats;

/* Algorithm 3 for the smoothed risk-averse problem: x (device, the linear-
 * quadratic layout; in: the initial guess, out: (y, u, p~) with the adjoint
 * scaled by zeta_j as for the linear-quadratic systems), f (device: its U and P
 * blocks are the problem's f_U and M f; its Y block is not read), yd (device
 * [n][n]: the target), *t (host; in: t^0, out: t).  The context's blocks give
 * A_j, D_j, E_j and G = nu M; its C_j are overwritten (c_j = zeta_j g'(Q_j)
 * mass / (1 - lambda)) and the rank-one terms are cleared on return.  F_1(x; t)
 * is S(c) x - [c_j y_d | f_U | f_P]; every Newton system J_11 dx = -F_1 and the
 * solve for F'(t) = J_22 - J_21 J_11^{-1} J_12 run GMRES preconditioned by one
 * V-cycle of S(c) from zero.  h(t) is computed by Newton from the current x with
 * a backtracking on ||F_1||, stopped by the rule of the risk-averse experiments
 * (Section 6): max(||F_1(x^k)|| / ||F_1(x^0)||, ||F_1(x^k)||) <= inner_tol
 * (inner_rule and inner_full_steps select the variants); when every g''(Q_j) vanishes (eq. condition) the step
 * is the split one (h(t^k), the root of F_2(x; t) = 0 by bisection, h at that
 * root); else
 * the Newton step on t with backtracking |F(t + gamma d)| - |F(t)| <=
 * -sigma |F(t)| (gamma = 1, rho, rho^2, ..., at most 30 reductions).  Needs
 * SMG_FLAG_CVAR and an FP64 context.  Returns SMG_OK, SMG_NOT_CONVERGED or an
 * error. */
int smg_cvar_solve(smg_ctx *ctx, double *x, const double *f, const double *yd, double *t,
                   const smg_cvar_params *prm, smg_cvar_stats *stats);

/* ------------------------------------------------------------------ batches
 * Many independent problem instances (different n, N and blocks) solved
 * together.  The smallest instances (a correction cycle touching at most 16 MB)
 * form one group, the others one group per finest grid size, and the groups
 * run one after another (smallest first) on the contexts' stream, so small
 * instances retire early.  Within a group every refinement step of all unretired
 * instances -- FP64 residual r_i = f_i - S_i x_i, convergence check, one
 * correction V-cycle from zero in the contexts' precision (red-black collective
 * Gauss-Seidel V(pre,post), Alg. 1), x_i += correction -- is one fixed sequence
 * of batched launches, each covering one phase of the group's instances at the
 * same hierarchy depth, captured once into a hipGraph and replayed.  An instance
 * is retired on the device as soon as its relative residual meets the
 * tolerance; its blocks then exit at once.  The instances' contexts must share
 * precision, pre, post and stream and use theta = 1 (pre, post >= 1).  Calls
 * that overlap on the same contexts race (the batch uses their scratch
 * buffers). */
typedef struct smg_batch smg_batch;

/* Device workspace bytes a batch over these contexts needs (0 if invalid). */
size_t smg_batch_workspace_bytes(smg_ctx *const *ctxs, int count);

/* Bind the instances' FP64 device vectors x[i] (initial guess in, solution
 * out) and f[i] to a batch.  lanes (host, may be NULL): lanes per grid node of
 * each instance (power of two <= 64 with at most 8 samples per lane), e.g. from
 * smg_tune_lanes; NULL picks the single-instance width: min(64, pow2ceil(N)),
 * or min(64, pow2ceil(N/2)) for an SMG_F32 context with even N (whose FP32
 * kernels take two consecutive samples per access when every instance's N is
 * even).  Computes ||f_i|| and
 * copies the launch tables into the workspace (>= smg_batch_workspace_bytes,
 * 256-byte aligned, caller-owned). */
int smg_batch_setup(smg_ctx *const *ctxs, int count, double *const *x, const double *const *f,
                    const int *lanes, void *workspace, size_t workspace_bytes, smg_batch **out);

/* Run refinement steps until every instance has ||f_i - S_i x_i||_2 <=
 * rtol ||f_i||_2 or has used maxit correction cycles.  stats (host, may be
 * NULL): count entries; iterations = correction cycles, relres, time_ms =
 * device time from the start of the call to the step that retired the
 * instance.  wall_ms (may be NULL): host wall time of the call.  Returns
 * SMG_NOT_CONVERGED if any instance hit maxit. */
int smg_batch_solve(smg_batch *batch, double rtol, int maxit, smg_stats *stats, double *wall_ms);

void smg_batch_destroy(smg_batch *batch);
const char *smg_batch_last_error(const smg_batch *batch);

/* Autotuner of the lanes-per-node width of the batched half-sweep for one
 * context: times the finest-level red half-sweep for each power-of-two width W
 * up to the default one (see smg_batch_setup) with at most 8 samples per lane,
 * with HIP events on the
 * context's stream.  lanes/us (host, cap entries) receive the candidates and
 * their average launch time in microseconds, *ncand their number, *best the
 * fastest width.  Overwrites the context's scratch vectors. */
int smg_tune_lanes(smg_ctx *ctx, int cap, int *lanes, double *us, int *ncand, int *best);

/* ------------------------------------------------------- warm-start network
 * A convolutional encoder-decoder (4 levels, 16/32/48/48 channels, nearest
 * upsampling with additive skips, SiLU, about 165k parameters) maps per-node
 * features of an instance -- mean and standard deviation over the samples of
 * the node log-coefficient, the target state y_d and log10(nu) + 4 -- on an
 * H x H grid (H a multiple of 8, H >= n, zero beyond the instance's nodes) to
 * a normalized prediction of (u, mean_j y_j, mean_j p_j).  Convolutions run as
 * implicit GEMMs on the BF16 matrix cores with FP32 accumulation; master
 * weights, gradients and Adam moments are FP32.  The prediction lifted to
 * x0 = (y_j = mean y, u, p_j = mean p) is an initial guess for smg_solve; the
 * caller keeps the zero start when ||f - S x0|| exceeds ||f||.
 * Parameters: one FP32 vector, per layer W[cout][tap][cin] (tap = 3 ky + kx)
 * followed by b[cout].  All tensors are device memory, NHWC, batch-major. */
typedef struct smg_net smg_net;

int smg_net_param_count(void);
/* workspace bytes for mini-batches of `batch` samples on an H x H grid (0 if invalid) */
size_t smg_net_workspace_bytes(int batch, int H);
int smg_net_setup(int batch, int H, void *workspace, size_t workspace_bytes, void *stream, smg_net **out);
void smg_net_destroy(smg_net *net);
const char *smg_net_last_error(const smg_net *net);
/* copy FP32 parameters in (resets the Adam state) / out */
int smg_net_set_params(smg_net *net, const float *theta);
int smg_net_get_params(smg_net *net, float *theta);
/* out[batch][H][H][3] (FP32) = network(x[batch][H][H][4] FP32) */
int smg_net_forward(smg_net *net, const float *x, float *out);
/* forward + backward of the mean squared error over pixels with y, x < valid
 * and the three channels: grad (device, param_count FP32, may be NULL) and
 * *loss (host, may be NULL); synchronizes the stream when loss is requested */
int smg_net_grad(smg_net *net, const float *x, const float *target, int valid, float *grad, float *loss);
/* forward + backward + one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) */
int smg_net_train_step(smg_net *net, const float *x, const float *target, int valid, float lr, float *loss);

/* features feat[H][H][4] of the instance behind ctx with right-hand side f */
int smg_net_features(smg_ctx *ctx, const double *f, int H, float *feat);
/* normalized targets tgt[H][H][3] from a solution x; norm (host) = {mean[3], std[3]} */
int smg_net_targets(smg_ctx *ctx, const double *x, int H, const float *norm, float *tgt);
/* x0 (device, ctx layout) from a normalized prediction pred[H][H][3] */
int smg_net_lift(smg_ctx *ctx, const float *pred, int H, const float *norm, double *x0);

#ifdef __cplusplus
}
#endif

#endif /* SMG_H */
