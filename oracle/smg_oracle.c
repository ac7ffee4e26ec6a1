/* smg_oracle.c -- plain CPU oracle of the collective multigrid method.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU path.  Everything is plain loops in FP64 (plus an FP32 copy
 * of the level operations, used as the reference of the mixed-precision
 * solver); nothing is blocked, fused or reordered beyond what the method
 * states.
 *
 * What it follows (Ciaramella, Nobile, Vanzan, "A collective multigrid ...",
 * arXiv 2302.13680):
 *   - the block system S x = f, eq. (2) and eq. full_space_optimality_system;
 *   - the node solve, eq. solution_reduced_system (Section 3);
 *   - the collective smoother, eq. collective_smoothing, in its Gauss-Seidel
 *     variant visited red then black (Section 3 allows Gauss-Seidel variants);
 *   - Alg. 1 (V-cycle) with a direct solve on the coarsest level;
 *   - GMRES preconditioned by one V-cycle (Section 3.2, experiments);
 *   - coarse operators by rediscretization (Section 3 allows it in place of
 *     the Galerkin product): face coefficients averaged pairwise, mass-type
 *     diagonal blocks scaled by 4 per level (they carry h^2).
 * The layout is the paper's (see oracle_levelops.h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REAL double
#define SFX(name) name##_f64
#include "oracle_levelops.h"
#undef REAL
#undef SFX
#define REAL float
#define SFX(name) name##_f32
#include "oracle_levelops.h"
#undef REAL
#undef SFX

#define OR_MAXLEV 16

typedef struct {
  int nlev, N, pre, post;
  double theta;
  int smoother;   /* 0: red-black collective Gauss-Seidel, 1: damped collective Jacobi */
  double *md[OR_MAXLEV], *me[OR_MAXLEV];   /* node factors of D_j, E_j per level (NULL: 1) */
  float *md32[OR_MAXLEV], *me32[OR_MAXLEV];
  double *dom[OR_MAXLEV];                  /* domain per level (NULL: the whole square) */
  float *dom32[OR_MAXLEV];
  int n[OR_MAXLEV];
  double *kx[OR_MAXLEV], *ky[OR_MAXLEV];
  double *c[OR_MAXLEV], *d[OR_MAXLEV], *e[OR_MAXLEV];
  double g[OR_MAXLEV];
  float *kx32[OR_MAXLEV], *ky32[OR_MAXLEV];
  float *c32[OR_MAXLEV], *d32[OR_MAXLEV], *e32[OR_MAXLEV];
  or_lvl_f64 L[OR_MAXLEV];
  or_lvl_f32 L32[OR_MAXLEV];
  double *xw[OR_MAXLEV], *fw[OR_MAXLEV], *rw[OR_MAXLEV];
  float *xw32[OR_MAXLEV], *fw32[OR_MAXLEV], *rw32[OR_MAXLEV];
  int m;          /* unknowns per field on the coarsest grid */
  double *Ainv;   /* [N][m][m] inverses of the coarsest A_j */
  double *Sinv;   /* [m][m] inverse of the coarsest control Schur complement */
  double *cw;     /* coarse-solve scratch */
} or_ctx;

static size_t vlen(int n, int N) { return (size_t)(2 * N + 1) * n * n; }

/* ---------------------------------------------------------------- dense LU */
/* Inverse of a dense m x m matrix by Gaussian elimination with partial pivoting
 * applied to [A | I].  Returns 0 on success, -1 on a zero pivot. */
static int or_dense_inverse(int m, const double *A, double *Ainv) {
  double *W = (double *)malloc(sizeof(double) * (size_t)m * 2 * m);
  int w = 2 * m;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < w; ++j)
      W[(size_t)i * w + j] = j < m ? A[(size_t)i * m + j] : (j - m == i ? 1.0 : 0.0);
  for (int col = 0; col < m; ++col) {
    int piv = col;
    for (int i = col + 1; i < m; ++i)
      if (fabs(W[(size_t)i * w + col]) > fabs(W[(size_t)piv * w + col])) piv = i;
    if (W[(size_t)piv * w + col] == 0.0) { free(W); return -1; }
    if (piv != col)
      for (int j = 0; j < w; ++j) {
        double t = W[(size_t)col * w + j];
        W[(size_t)col * w + j] = W[(size_t)piv * w + j];
        W[(size_t)piv * w + j] = t;
      }
    double dv = W[(size_t)col * w + col];
    for (int j = 0; j < w; ++j) W[(size_t)col * w + j] /= dv;
    for (int i = 0; i < m; ++i) {
      if (i == col) continue;
      double fct = W[(size_t)i * w + col];
      if (fct == 0.0) continue;
      for (int j = 0; j < w; ++j) W[(size_t)i * w + j] -= fct * W[(size_t)col * w + j];
    }
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) Ainv[(size_t)i * m + j] = W[(size_t)i * w + m + j];
  free(W);
  return 0;
}

static void matvec(int m, const double *A, const double *v, double *out) {
  for (int i = 0; i < m; ++i) {
    double s = 0;
    for (int j = 0; j < m; ++j) s += A[(size_t)i * m + j] * v[j];
    out[i] = s;
  }
}

/* ------------------------------------------------------------- hierarchy */
/* Coarse faces (rediscretization): the coarse x-face between coarse nodes X-1
 * and X on coarse row K spans the two fine x-faces 2X and 2X+1 of fine row
 * 2K+1; its coefficient is their mean.  Likewise for y-faces. */
void or_coarsen_faces(int nf, int N, const double *kxf, const double *kyf,
                      double *kxc, double *kyc) {
  int nc = (nf - 1) / 2;
  for (int j = 0; j < N; ++j) {
    for (int K = 0; K < nc; ++K)
      for (int F = 0; F <= nc; ++F)
        kxc[((size_t)j * nc + K) * (nc + 1) + F] =
            0.5 * (kxf[((size_t)j * nf + 2 * K + 1) * (nf + 1) + 2 * F] +
                   kxf[((size_t)j * nf + 2 * K + 1) * (nf + 1) + 2 * F + 1]);
    for (int G = 0; G <= nc; ++G)
      for (int X = 0; X < nc; ++X)
        kyc[((size_t)j * (nc + 1) + G) * nc + X] =
            0.5 * (kyf[((size_t)j * (nf + 1) + 2 * G) * nf + 2 * X + 1] +
                   kyf[((size_t)j * (nf + 1) + 2 * G + 1) * nf + 2 * X + 1]);
  }
}

/* Direct solver of the coarsest level (Alg. 1, first branch), by block
 * elimination of eq. (2): eliminating y_j and p_j through A_j leaves the
 * control Schur complement  G + sum_j D_j A_j^{-1} C_j A_j^{-1} E_j  (the
 * matrix counterpart of the denominator in eq. solution_reduced_system). */
static int or_coarse_setup(or_ctx *C) {
  int l = C->nlev - 1, n = C->n[l], N = C->N, m = n * n;
  C->m = m;
  C->Ainv = (double *)malloc(sizeof(double) * (size_t)N * m * m);
  C->Sinv = (double *)malloc(sizeof(double) * (size_t)m * m);
  C->cw = (double *)malloc(sizeof(double) * (size_t)m * 4);
  double *A = (double *)malloc(sizeof(double) * (size_t)m * m);
  double *Sch = (double *)calloc((size_t)m * m, sizeof(double));
  double *e_i = (double *)calloc((size_t)m, sizeof(double));
  double *col = (double *)malloc(sizeof(double) * (size_t)m);
  or_lvl_f64 *L = &C->L[l];
  for (int i = 0; i < m; ++i) Sch[(size_t)i * m + i] = L->g;
  /* with node factors, D_j = d_j diag(md) and E_j = e_j diag(me) (0 outside the domain) */
  for (int j = 0; j < N; ++j) {
    /* assemble A_j column by column from the stencil; nodes outside the domain
     * get identity rows (their couplings vanish: the stencil reads them as 0) */
    for (int q = 0; q < m; ++q) {
      memset(e_i, 0, sizeof(double) * m);
      e_i[q] = 1.0;
      for (int k = 0; k < n; ++k)
        for (int x = 0; x < n; ++x) A[(size_t)(k * n + x) * m + q] = or_stencil_f64(L, j, e_i, x, k);
    }
    for (int r = 0; r < m; ++r)
      if (!or_live_f64(L, (size_t)r)) {
        for (int q = 0; q < m; ++q) A[(size_t)r * m + q] = 0.0;
        A[(size_t)r * m + r] = 1.0;
      }
    double *Ai = C->Ainv + (size_t)j * m * m;
    if (or_dense_inverse(m, A, Ai) != 0) goto fail;
    /* Sch += d_j c_j e_j Ainv_j Ainv_j */
    double s = L->d[j] * L->c[j] * L->e[j];
    for (int q = 0; q < m; ++q) {
      for (int i = 0; i < m; ++i) col[i] = Ai[(size_t)i * m + q];
      for (int i = 0; i < m; ++i) {
        double t = 0;
        for (int r = 0; r < m; ++r) t += Ai[(size_t)i * m + r] * col[r];
        Sch[(size_t)i * m + q] += (or_mask_d_f64(L, (size_t)i) * s * or_mask_e_f64(L, (size_t)q)) * t;
      }
    }
  }
  if (or_dense_inverse(m, Sch, C->Sinv) != 0) goto fail;
  free(A); free(Sch); free(e_i); free(col);
  return 0;
fail:
  free(A); free(Sch); free(e_i); free(col);
  return -1;
}

/* X = S_coarsest^{-1} F (block layout of eq. (2)). */
void or_coarse_solve(const or_ctx *C, const double *F, double *X) {
  int l = C->nlev - 1, m = C->m, N = C->N;
  const or_lvl_f64 *L = &C->L[l];
  double *rhs = C->cw, *t1 = C->cw + m, *t2 = C->cw + 2 * m, *uu = C->cw + 3 * m;
  for (int i = 0; i < m; ++i) rhs[i] = F[(size_t)N * m + i];
  for (int j = 0; j < N; ++j) {
    const double *Ai = C->Ainv + (size_t)j * m * m;
    const double *FY = F + (size_t)j * m, *FP = F + (size_t)(N + 1) * m + (size_t)j * m;
    matvec(m, Ai, FP, t1);                                        /* A^{-1} F_P */
    for (int i = 0; i < m; ++i) t2[i] = FY[i] - L->c[j] * t1[i];
    matvec(m, Ai, t2, t1);                                        /* A^{-1}(F_Y - C A^{-1} F_P) */
    for (int i = 0; i < m; ++i) rhs[i] -= (or_mask_d_f64(L, i) * L->d[j]) * t1[i];
  }
  matvec(m, C->Sinv, rhs, uu);
  for (int i = 0; i < m; ++i) X[(size_t)N * m + i] = uu[i];
  for (int j = 0; j < N; ++j) {
    const double *Ai = C->Ainv + (size_t)j * m * m;
    const double *FY = F + (size_t)j * m, *FP = F + (size_t)(N + 1) * m + (size_t)j * m;
    double *Y = X + (size_t)j * m, *P = X + (size_t)(N + 1) * m + (size_t)j * m;
    for (int i = 0; i < m; ++i) t2[i] = FP[i] - (or_mask_e_f64(L, i) * L->e[j]) * uu[i];
    matvec(m, Ai, t2, Y);                                         /* y = A^{-1}(F_P - E u) */
    for (int i = 0; i < m; ++i) t2[i] = FY[i] - L->c[j] * Y[i];
    matvec(m, Ai, t2, P);                                         /* p = A^{-1}(F_Y - C y) */
  }
}

void or_destroy(or_ctx *C) {
  if (!C) return;
  for (int l = 0; l < C->nlev; ++l) {
    free(C->kx[l]); free(C->ky[l]); free(C->c[l]); free(C->d[l]); free(C->e[l]);
    free(C->kx32[l]); free(C->ky32[l]); free(C->c32[l]); free(C->d32[l]); free(C->e32[l]);
    free(C->xw[l]); free(C->fw[l]); free(C->rw[l]);
    free(C->xw32[l]); free(C->fw32[l]); free(C->rw32[l]);
  }
  for (int l = 0; l < C->nlev; ++l) { free(C->md[l]); free(C->md32[l]); free(C->me[l]); free(C->me32[l]); }
  for (int l = 0; l < C->nlev; ++l) { free(C->dom[l]); free(C->dom32[l]); }
  free(C->Ainv); free(C->Sinv); free(C->cw);
  free(C);
}

static float *to_f32(const double *v, size_t len) {
  float *o = (float *)malloc(sizeof(float) * len);
  for (size_t i = 0; i < len; ++i) o[i] = (float)v[i];
  return o;
}

/* Build the level hierarchy n -> (n-1)/2 down to coarsest_n.  Returns NULL if
 * n is not of the form (coarsest_n+1) 2^k - 1 or a coarsest block is singular. */
or_ctx *or_create(int n, int N, int coarsest_n, int pre, int post, double theta,
                  const double *kx, const double *ky, const double *c, const double *d,
                  const double *e, double g) {
  if (n < 1 || N < 1 || coarsest_n < 1) return NULL;
  int nlev = 1, t = n;
  while (t > coarsest_n) {
    if ((t & 1) == 0) return NULL;
    t = (t - 1) / 2;
    ++nlev;
    if (nlev > OR_MAXLEV) return NULL;
  }
  if (t != coarsest_n) return NULL;
  or_ctx *C = (or_ctx *)calloc(1, sizeof(or_ctx));
  C->nlev = nlev; C->N = N; C->pre = pre; C->post = post; C->theta = theta;
  for (int l = 0; l < nlev; ++l) {
    int nl = l == 0 ? n : (C->n[l - 1] - 1) / 2;
    C->n[l] = nl;
    size_t fx = (size_t)N * nl * (nl + 1);
    C->kx[l] = (double *)malloc(sizeof(double) * fx);
    C->ky[l] = (double *)malloc(sizeof(double) * fx);
    C->c[l] = (double *)malloc(sizeof(double) * N);
    C->d[l] = (double *)malloc(sizeof(double) * N);
    C->e[l] = (double *)malloc(sizeof(double) * N);
    if (l == 0) {
      memcpy(C->kx[l], kx, sizeof(double) * fx);
      memcpy(C->ky[l], ky, sizeof(double) * fx);
      memcpy(C->c[l], c, sizeof(double) * N);
      memcpy(C->d[l], d, sizeof(double) * N);
      memcpy(C->e[l], e, sizeof(double) * N);
      C->g[l] = g;
    } else {
      or_coarsen_faces(C->n[l - 1], N, C->kx[l - 1], C->ky[l - 1], C->kx[l], C->ky[l]);
      for (int j = 0; j < N; ++j) {
        C->c[l][j] = 4.0 * C->c[l - 1][j];
        C->d[l][j] = 4.0 * C->d[l - 1][j];
        C->e[l][j] = 4.0 * C->e[l - 1][j];
      }
      C->g[l] = 4.0 * C->g[l - 1];
    }
    C->kx32[l] = to_f32(C->kx[l], fx);
    C->ky32[l] = to_f32(C->ky[l], fx);
    C->c32[l] = to_f32(C->c[l], N);
    C->d32[l] = to_f32(C->d[l], N);
    C->e32[l] = to_f32(C->e[l], N);
    or_lvl_f64 L = {nl, N, C->kx[l], C->ky[l], C->c[l], C->d[l], C->e[l], C->g[l]};
    or_lvl_f32 L32 = {nl, N, C->kx32[l], C->ky32[l], C->c32[l], C->d32[l], C->e32[l], (float)C->g[l]};
    C->L[l] = L;
    C->L32[l] = L32;
    size_t len = vlen(nl, N);
    C->xw[l] = (double *)calloc(len, sizeof(double));
    C->fw[l] = (double *)calloc(len, sizeof(double));
    C->rw[l] = (double *)calloc(len, sizeof(double));
    C->xw32[l] = (float *)calloc(len, sizeof(float));
    C->fw32[l] = (float *)calloc(len, sizeof(float));
    C->rw32[l] = (float *)calloc(len, sizeof(float));
  }
  if (or_coarse_setup(C) != 0) { or_destroy(C); return NULL; }
  return C;
}

/* Per-level copies of a finest-level node factor, level by level: coarse node
 * (X, K) takes the value of fine node (2X+1, 2K+1) (coarsen 0: injection) or
 * the full-weighting average of the 3 x 3 fine nodes around it, weights
 * (1/4)(1/2)^(|dx|+|dk|) (coarsen 1: the diagonal of the Galerkin product
 * R diag(v) P lumped by rows, R = P^T / 4).  src NULL: all levels NULL. */
static void set_factor(or_ctx *C, const double *src, double **lv, float **lv32, int coarsen) {
  for (int l = 0; l < C->nlev; ++l) {
    free(lv[l]); free(lv32[l]);
    lv[l] = NULL; lv32[l] = NULL;
  }
  if (!src) return;
  for (int l = 0; l < C->nlev; ++l) {
    int nl = C->n[l];
    lv[l] = (double *)malloc(sizeof(double) * (size_t)nl * nl);
    if (l == 0) {
      memcpy(lv[0], src, sizeof(double) * (size_t)nl * nl);
    } else {
      int nf = C->n[l - 1];
      for (int K = 0; K < nl; ++K)
        for (int X = 0; X < nl; ++X) {
          const double *F = lv[l - 1];
          if (!coarsen) {
            lv[l][(size_t)K * nl + X] = F[(size_t)(2 * K + 1) * nf + 2 * X + 1];
            continue;
          }
          double acc = 0.0;
          for (int dk = -1; dk <= 1; ++dk)
            for (int dx = -1; dx <= 1; ++dx)
              acc += (dx ? 0.5 : 1.0) * (dk ? 0.5 : 1.0) * 0.25 * F[(size_t)(2 * K + 1 + dk) * nf + 2 * X + 1 + dx];
          lv[l][(size_t)K * nl + X] = acc;
        }
    }
    lv32[l] = to_f32(lv[l], (size_t)nl * nl);
  }
}

/* Node factors of D_j and E_j: the node entries become md_i d_j and me_i e_j on
 * every level, coarse factors by injection (coarsen 0) or full weighting
 * (coarsen 1); the coarsest factorization is rebuilt.  md, me: [n][n] of the
 * finest level, or NULL for 1 everywhere.  Returns 0, or -1 if the coarsest
 * system is singular. */
int or_set_masks(or_ctx *C, const double *md, const double *me, int coarsen) {
  set_factor(C, md, C->md, C->md32, coarsen);
  set_factor(C, me, C->me, C->me32, coarsen);
  for (int l = 0; l < C->nlev; ++l) {
    C->L[l].md = C->md[l]; C->L32[l].md = C->md32[l];
    C->L[l].me = C->me[l]; C->L32[l].me = C->me32[l];
  }
  free(C->Ainv); free(C->Sinv); free(C->cw);
  C->Ainv = C->Sinv = C->cw = NULL;
  return or_coarse_setup(C);
}

/* The domain: dom [n][n] of the finest level, 1 inside, 0 outside (NULL: the
 * whole square).  Nodes outside are homogeneous Dirichlet nodes held at zero;
 * coarse levels by injection, which keeps the domain exactly when its edges
 * lie on grid lines of every level (the L-shape (0,1)^2 minus [1/2,1)^2 does).
 * The coarsest factorization is rebuilt.  Returns 0, or -1 if singular. */
int or_set_domain(or_ctx *C, const double *dom) {
  set_factor(C, dom, C->dom, C->dom32, 0);
  for (int l = 0; l < C->nlev; ++l) { C->L[l].dom = C->dom[l]; C->L32[l].dom = C->dom32[l]; }
  free(C->Ainv); free(C->Sinv); free(C->cw);
  C->Ainv = C->Sinv = C->cw = NULL;
  return or_coarse_setup(C);
}

/* Per-sample state-mass values c_j of the finest level (c_j >= 0; the Y-block
 * blocks C_j = c_j I of the risk-averse Newton systems, Section 6): level l
 * takes 4^l c_j, as at creation.  The coarsest factorization is rebuilt.
 * Returns 0, -1 if a value is negative or the coarsest block singular. */
int or_set_sample_c(or_ctx *C, const double *c) {
  for (int j = 0; j < C->N; ++j)
    if (!(c[j] >= 0.0)) return -1;
  for (int l = 0; l < C->nlev; ++l)
    for (int j = 0; j < C->N; ++j) {
      C->c[l][j] = l == 0 ? c[j] : 4.0 * C->c[l - 1][j];
      C->c32[l][j] = (float)C->c[l][j];
    }
  free(C->Ainv); free(C->Sinv); free(C->cw);
  C->Ainv = C->Sinv = C->cw = NULL;
  return or_coarse_setup(C);
}

/* Rediscretized control blocks for a control on a line: D_j, E_j and G of level
 * l >= 1 become growth^l times the finest ones (growth 2: the 1D mass of the
 * control line doubles with the spacing; or_create's default 4 is the h^2 of an
 * area mass, as for C_j).  The coarsest factorization is rebuilt.  Returns 0,
 * -1 if singular or growth is not positive. */
int or_set_control_growth(or_ctx *C, double growth) {
  if (!(growth > 0.0)) return -1;
  for (int l = 1; l < C->nlev; ++l) {
    for (int j = 0; j < C->N; ++j) {
      C->d[l][j] = growth * C->d[l - 1][j];
      C->e[l][j] = growth * C->e[l - 1][j];
      C->d32[l][j] = (float)C->d[l][j];
      C->e32[l][j] = (float)C->e[l][j];
    }
    C->g[l] = growth * C->g[l - 1];
    C->L[l].g = C->g[l];
    C->L32[l].g = (float)C->g[l];
  }
  free(C->Ainv); free(C->Sinv); free(C->cw);
  C->Ainv = C->Sinv = C->cw = NULL;
  return or_coarse_setup(C);
}

/* Control acting only where mask[i] != 0 (local control; eq.
 * solution_reduced_system2 at nodes without control): the node entries of D_j
 * and E_j become mask_i d_j and mask_i e_j.  mask NULL: control everywhere. */
int or_set_control(or_ctx *C, const double *mask) { return or_set_masks(C, mask, mask, 0); }

/* The node factor of every level (after or_set_masks): out [n_l][n_l], 1 where
 * the factor is absent.  which 0: md, 1: me. */
void or_level_factor(const or_ctx *C, int l, int which, double *out) {
  const double *v = which ? C->me[l] : C->md[l];
  size_t nn = (size_t)C->n[l] * C->n[l];
  for (size_t i = 0; i < nn; ++i) out[i] = v ? v[i] : 1.0;
}

/* The domain of level l: out [n_l][n_l], 1 inside (everywhere without one). */
void or_level_domain(const or_ctx *C, int l, double *out) {
  size_t nn = (size_t)C->n[l] * C->n[l];
  for (size_t i = 0; i < nn; ++i) out[i] = C->dom[l] ? C->dom[l][i] : 1.0;
}

int or_nlevels(const or_ctx *C) { return C->nlev; }
int or_level_n(const or_ctx *C, int l) { return C->n[l]; }
void or_level_faces(const or_ctx *C, int l, double *kx, double *ky) {
  size_t fx = (size_t)C->N * C->n[l] * (C->n[l] + 1);
  memcpy(kx, C->kx[l], sizeof(double) * fx);
  memcpy(ky, C->ky[l], sizeof(double) * fx);
}
void or_level_scalars(const or_ctx *C, int l, double *c, double *d, double *e, double *g) {
  memcpy(c, C->c[l], sizeof(double) * C->N);
  memcpy(d, C->d[l], sizeof(double) * C->N);
  memcpy(e, C->e[l], sizeof(double) * C->N);
  *g = C->g[l];
}

/* --------------------------------------------------------- exported steps */
void or_apply(const or_ctx *C, int l, const double *x, double *out) { or_apply_f64(&C->L[l], x, out); }
void or_residual(const or_ctx *C, int l, const double *x, const double *f, double *r) {
  or_residual_f64(&C->L[l], x, f, r);
}
void or_halfsweep(const or_ctx *C, int l, int colour, double theta, double *x, const double *f) {
  or_halfsweep_f64(&C->L[l], colour, theta, x, f);
}
void or_jacobi(const or_ctx *C, int l, double theta, double *x, const double *f) {
  or_jacobi_f64(&C->L[l], theta, x, f);
}
void or_restrict(int nf, int N, const double *fine, double *coarse) { or_restrict_f64(nf, N, fine, coarse); }
void or_prolong_add(int nc, int N, const double *coarse, double *fine) { or_prolong_add_f64(nc, N, coarse, fine, NULL); }
/* The coarse right-hand side of Alg. 1 from level l: R (f - S x) with the U
 * block restricted within the control space, zero outside the domain. */
void or_residual_restrict(or_ctx *C, int l, const double *x, const double *f, double *coarse) {
  or_residual_f64(&C->L[l], x, f, C->rw[l]);
  control_residual_f64(&C->L[l], C->rw[l]);
  or_restrict_f64(C->n[l], C->N, C->rw[l], coarse);
  control_coarse_rows_f64(&C->L[l], C->n[l + 1], coarse);
  zero_outside_f64(&C->L[l + 1], coarse);
}
/* fine (level l) += P coarse, the U block into the control space only. */
void or_prolong_control(const or_ctx *C, int l, const double *coarse, double *fine) {
  or_prolong_add_f64(C->n[l + 1], C->N, coarse, fine, &C->L[l]);
}
void or_node_solve(int N, const double *a, const double *c, const double *d, const double *e, double g,
                   const double *bP, double bU, const double *bY, double *y, double *u, double *p) {
  or_node_solve_f64(N, a, c, d, e, g, bP, bU, bY, y, u, p);
}

/* --------------------------------------------------------------- V-cycle */
/* One smoothing step: a collective Gauss-Seidel sweep (red then black
 * half-sweeps) or a damped collective Jacobi step (eq. collective_smoothing). */
static void smooth_f64(const or_ctx *C, const or_lvl_f64 *L, double *x, const double *f) {
  if (C->smoother == 1) {
    or_jacobi_f64(L, C->theta, x, f);
  } else {
    or_halfsweep_f64(L, 0, C->theta, x, f);
    or_halfsweep_f64(L, 1, C->theta, x, f);
  }
}
static void smooth_f32(const or_ctx *C, const or_lvl_f32 *L, float *x, const float *f) {
  float th = (float)C->theta;
  if (C->smoother == 1) {
    or_jacobi_f32(L, th, x, f);
  } else {
    or_halfsweep_f32(L, 0, th, x, f);
    or_halfsweep_f32(L, 1, th, x, f);
  }
}

/* Set the smoother of the context's V-cycles: 0 = collective Gauss-Seidel
 * (default), 1 = damped collective Jacobi with damping theta. */
void or_set_smoother(or_ctx *C, int smoother) { C->smoother = smoother; }

/* Alg. 1 with n1 = pre and n2 = post smoothing steps, residual, restriction,
 * recursive call from a zero initial guess, coarse correction, post-smoothing. */
static void vcycle_f64(or_ctx *C, int l, double *x, const double *f) {
  if (l == C->nlev - 1) { or_coarse_solve(C, f, x); return; }
  const or_lvl_f64 *L = &C->L[l];
  for (int s = 0; s < C->pre; ++s) smooth_f64(C, L, x, f);
  or_residual_f64(L, x, f, C->rw[l]);
  control_residual_f64(L, C->rw[l]);
  or_restrict_f64(C->n[l], C->N, C->rw[l], C->fw[l + 1]);
  control_coarse_rows_f64(L, C->n[l + 1], C->fw[l + 1]);
  zero_outside_f64(&C->L[l + 1], C->fw[l + 1]);
  memset(C->xw[l + 1], 0, sizeof(double) * vlen(C->n[l + 1], C->N));
  vcycle_f64(C, l + 1, C->xw[l + 1], C->fw[l + 1]);
  or_prolong_add_f64(C->n[l + 1], C->N, C->xw[l + 1], x, L);
  for (int s = 0; s < C->post; ++s) smooth_f64(C, L, x, f);
}

/* The same cycle in FP32 arithmetic; the coarsest direct solve stays FP64. */
static void vcycle_f32(or_ctx *C, int l, float *x, const float *f) {
  int N = C->N;
  if (l == C->nlev - 1) {
    size_t len = vlen(C->n[l], N);
    double *F = (double *)malloc(sizeof(double) * len), *X = (double *)malloc(sizeof(double) * len);
    for (size_t i = 0; i < len; ++i) F[i] = (double)f[i];
    or_coarse_solve(C, F, X);
    for (size_t i = 0; i < len; ++i) x[i] = (float)X[i];
    free(F); free(X);
    return;
  }
  const or_lvl_f32 *L = &C->L32[l];
  for (int s = 0; s < C->pre; ++s) smooth_f32(C, L, x, f);
  or_residual_f32(L, x, f, C->rw32[l]);
  control_residual_f32(L, C->rw32[l]);
  or_restrict_f32(C->n[l], N, C->rw32[l], C->fw32[l + 1]);
  control_coarse_rows_f32(L, C->n[l + 1], C->fw32[l + 1]);
  zero_outside_f32(&C->L32[l + 1], C->fw32[l + 1]);
  memset(C->xw32[l + 1], 0, sizeof(float) * vlen(C->n[l + 1], N));
  vcycle_f32(C, l + 1, C->xw32[l + 1], C->fw32[l + 1]);
  or_prolong_add_f32(C->n[l + 1], N, C->xw32[l + 1], x, L);
  for (int s = 0; s < C->post; ++s) smooth_f32(C, L, x, f);
}

void or_vcycle(or_ctx *C, double *x, const double *f, int ncycles) {
  for (int i = 0; i < ncycles; ++i) vcycle_f64(C, 0, x, f);
}

/* ncycles FP32 V-cycles on FP64 in/out buffers (inputs rounded to FP32). */
void or_vcycle32(or_ctx *C, double *x, const double *f, int ncycles) {
  size_t len = vlen(C->n[0], C->N);
  float *x32 = to_f32(x, len), *f32 = to_f32(f, len);
  for (int i = 0; i < ncycles; ++i) vcycle_f32(C, 0, x32, f32);
  for (size_t i = 0; i < len; ++i) x[i] = (double)x32[i];
  free(x32); free(f32);
}

/* One FP32 half-sweep of level l on FP64 in/out buffers (x and f rounded to
 * FP32 first, the result widened back): the reference of the FP32 smoother. */
void or_halfsweep32(const or_ctx *C, int l, int colour, double theta, double *x, const double *f) {
  size_t len = vlen(C->n[l], C->N);
  float *x32 = to_f32(x, len), *f32 = to_f32(f, len);
  or_halfsweep_f32(&C->L32[l], colour, (float)theta, x32, f32);
  for (size_t i = 0; i < len; ++i) x[i] = (double)x32[i];
  free(x32); free(f32);
}

/* threads the node loops run on (the CPU baseline reports it) */
int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* 2-norm with a fixed summation order. */
double or_norm(const double *v, size_t len) {
  double s = 0;
  for (size_t i = 0; i < len; ++i) s += v[i] * v[i];
  return sqrt(s);
}

static double dot(const double *a, const double *b, size_t len) {
  double s = 0;
  for (size_t i = 0; i < len; ++i) s += a[i] * b[i];
  return s;
}

/* Stationary iteration: repeat Alg. 1 until ||f - S x|| <= tol ||f|| (the
 * relative unpreconditioned residual of the experiments).  hist[k] holds the
 * relative residual after k cycles (hist[0] for the initial guess); returns the
 * number of cycles, or -1 if maxit was reached first. */
int or_solve_vcycle(or_ctx *C, double *x, const double *f, double tol, int maxit, double *hist) {
  size_t len = vlen(C->n[0], C->N);
  double *r = (double *)malloc(sizeof(double) * len);
  double fn = or_norm(f, len);
  or_residual_f64(&C->L[0], x, f, r);
  double rel = or_norm(r, len) / fn;
  if (hist) hist[0] = rel;
  int k = 0;
  while (rel > tol && k < maxit) {
    vcycle_f64(C, 0, x, f);
    ++k;
    or_residual_f64(&C->L[0], x, f, r);
    rel = or_norm(r, len) / fn;
    if (hist) hist[k] = rel;
  }
  free(r);
  return rel <= tol ? k : -1;
}

/* Right-preconditioned restarted GMRES(m) with modified Gram-Schmidt and
 * Givens rotations; the preconditioner is one V-cycle from a zero guess
 * (FP64 when prec32 == 0, the FP32 cycle otherwise).  Stops when the
 * recurrence residual reaches tol ||f||; the explicit residual is checked
 * at the end of every cycle and a new cycle starts if it is not below tol.
 * hist[k] = relative residual (recurrence) after k iterations.  Returns the
 * iteration count, or -1 at maxit. */
int or_gmres(or_ctx *C, double *x, const double *f, int m, double tol, int maxit, int prec32,
             double *hist) {
  size_t len = vlen(C->n[0], C->N);
  double *V = (double *)malloc(sizeof(double) * len * (m + 1));
  double *Z = (double *)malloc(sizeof(double) * len * m);
  double *w = (double *)malloc(sizeof(double) * len);
  double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
  double *cs = (double *)malloc(sizeof(double) * m), *sn = (double *)malloc(sizeof(double) * m);
  double *gv = (double *)malloc(sizeof(double) * (m + 1)), *yv = (double *)malloc(sizeof(double) * m);
  double fn = or_norm(f, len);
  int its = 0, converged = 0;
  or_residual_f64(&C->L[0], x, f, w);
  double beta = or_norm(w, len);
  if (hist) hist[0] = beta / fn;
  if (beta <= tol * fn) converged = 1;
  while (!converged && its < maxit) {
    for (size_t i = 0; i < len; ++i) V[i] = w[i] / beta;
    for (int i = 0; i <= m; ++i) gv[i] = 0;
    gv[0] = beta;
    int kend = 0;
    for (int k = 0; k < m; ++k) {
      double *vk = V + (size_t)k * len, *zk = Z + (size_t)k * len;
      memset(zk, 0, sizeof(double) * len);
      if (prec32) or_vcycle32(C, zk, vk, 1); else vcycle_f64(C, 0, zk, vk);
      or_apply_f64(&C->L[0], zk, w);
      for (int i = 0; i <= k; ++i) {
        double hik = dot(w, V + (size_t)i * len, len);
        H[(size_t)i * m + k] = hik;
        for (size_t q = 0; q < len; ++q) w[q] -= hik * V[(size_t)i * len + q];
      }
      double hn = or_norm(w, len);
      H[(size_t)(k + 1) * m + k] = hn;
      if (hn > 0)
        for (size_t q = 0; q < len; ++q) V[(size_t)(k + 1) * len + q] = w[q] / hn;
      for (int i = 0; i < k; ++i) {
        double a = H[(size_t)i * m + k], b = H[(size_t)(i + 1) * m + k];
        H[(size_t)i * m + k] = cs[i] * a + sn[i] * b;
        H[(size_t)(i + 1) * m + k] = -sn[i] * a + cs[i] * b;
      }
      double a = H[(size_t)k * m + k], b = H[(size_t)(k + 1) * m + k];
      double rr = sqrt(a * a + b * b);
      cs[k] = a / rr;
      sn[k] = b / rr;
      H[(size_t)k * m + k] = rr;
      H[(size_t)(k + 1) * m + k] = 0;
      gv[k + 1] = -sn[k] * gv[k];
      gv[k] = cs[k] * gv[k];
      ++its;
      kend = k + 1;
      if (hist) hist[its] = fabs(gv[k + 1]) / fn;
      if (fabs(gv[k + 1]) <= tol * fn || its >= maxit || hn == 0) break;
    }
    for (int i = kend - 1; i >= 0; --i) {
      double s = gv[i];
      for (int q = i + 1; q < kend; ++q) s -= H[(size_t)i * m + q] * yv[q];
      yv[i] = s / H[(size_t)i * m + i];
    }
    for (int i = 0; i < kend; ++i)
      for (size_t q = 0; q < len; ++q) x[q] += yv[i] * Z[(size_t)i * len + q];
    or_residual_f64(&C->L[0], x, f, w);
    beta = or_norm(w, len);
    if (beta <= tol * fn) converged = 1;
  }
  free(V); free(Z); free(w); free(H); free(cs); free(sn); free(gv); free(yv);
  return converged ? its : -1;
}

/* Mixed precision: FP64 iterative refinement.  Each outer step computes the
 * FP64 residual r = f - S x and a correction d from the FP32 V-cycle: with
 * m > 0, d comes from a flexible GMRES(m) cycle (FP64 Arnoldi and matvec, the
 * FP32 V-cycle as preconditioner) stopped at inner_tol relative to ||r||;
 * with m == 0, d is one FP32 V-cycle applied to r from a zero guess.  Then
 * x += d.  hist[k] = FP64 relative residual after k outer steps.  Returns the
 * number of outer steps (or -1 at maxit); *inner gets the total number of
 * inner GMRES iterations (the number of FP32 V-cycles). */
int or_solve_ir(or_ctx *C, double *x, const double *f, double tol, double inner_tol, int m,
                int maxit, double *hist, int *inner) {
  size_t len = vlen(C->n[0], C->N);
  double *r = (double *)malloc(sizeof(double) * len), *dd = (double *)malloc(sizeof(double) * len);
  double fn = or_norm(f, len);
  int k = 0, tot = 0;
  or_residual_f64(&C->L[0], x, f, r);
  double rel = or_norm(r, len) / fn;
  if (hist) hist[0] = rel;
  while (rel > tol && k < maxit) {
    memset(dd, 0, sizeof(double) * len);
    if (m > 0) {
      int it = or_gmres(C, dd, r, m, inner_tol, m, 1, NULL);
      tot += it < 0 ? m : it;
    } else {
      or_vcycle32(C, dd, r, 1);
      tot += 1;
    }
    for (size_t i = 0; i < len; ++i) x[i] += dd[i];
    ++k;
    or_residual_f64(&C->L[0], x, f, r);
    rel = or_norm(r, len) / fn;
    if (hist) hist[k] = rel;
  }
  if (inner) *inner = tot;
  free(r); free(dd);
  return rel <= tol ? k : -1;
}
