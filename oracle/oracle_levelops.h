/* Level operations of the CPU oracle, written once over a scalar type.
 *
 * TEST INFRASTRUCTURE: included twice by smg_oracle.c, once with REAL=double
 * (suffix _f64) and once with REAL=float (suffix _f32, the reduced-precision
 * V-cycle used as the reference of the mixed-precision solver).
 *
 * Vector layout is the paper's, eq. (2): x = [y_1 .. y_N | u | p_1 .. p_N],
 * every block an n x n grid stored row-major (row k slow, column x fast).
 * Faces: kx[j][k][f], f = 0..n, between columns f-1 and f of row k;
 *        ky[j][g][x], g = 0..n, between rows g-1 and g of column x.
 * Nodes outside the grid carry the value 0 (homogeneous Dirichlet).
 */

typedef struct {
  int n, N;
  const REAL *kx, *ky;       /* [N][n][n+1], [N][n+1][n] */
  const REAL *c, *d, *e;     /* [N] diagonal values of C_j, D_j, E_j */
  REAL g;                    /* diagonal value of G */
  const REAL *md, *me;       /* [n][n] node factors (NULL: 1 everywhere): the node entries
                                of D_j and E_j are md_i d_j and me_i e_j.  Local control:
                                md = me = the control mask; the semismooth Newton system
                                of Section 5: md = the active-set indicator, me = 1 */
  const REAL *dom;           /* [n][n] domain (NULL: the whole square): 0 marks a node
                                outside it (the L-shape's removed quadrant), a Dirichlet
                                node held at 0 whose rows of S are zero */
} SFX(or_lvl);

/* node i inside the domain */
static inline int SFX(or_live)(const SFX(or_lvl) *L, size_t i) { return !L->dom || L->dom[i] != (REAL)0; }

/* node factors of D_j and E_j at node i (0 outside the domain) */
static inline REAL SFX(or_mask_d)(const SFX(or_lvl) *L, size_t i) {
  return SFX(or_live)(L, i) ? (L->md ? L->md[i] : (REAL)1) : (REAL)0;
}
static inline REAL SFX(or_mask_e)(const SFX(or_lvl) *L, size_t i) {
  return SFX(or_live)(L, i) ? (L->me ? L->me[i] : (REAL)1) : (REAL)0;
}

#define OR_KX(L, j, k, f) ((L)->kx[((size_t)(j) * (L)->n + (k)) * ((L)->n + 1) + (f)])
#define OR_KY(L, j, gg, x) ((L)->ky[((size_t)(j) * ((L)->n + 1) + (gg)) * (L)->n + (x)])

/* value of grid function v (an n x n plane) at (x, k), zero outside the grid */
static inline REAL SFX(or_at)(const REAL *v, int n, int x, int k) {
  if (x < 0 || x >= n || k < 0 || k >= n) return (REAL)0;
  return v[(size_t)k * n + x];
}

/* the same, also zero outside the domain (homogeneous Dirichlet there) */
static inline REAL SFX(or_atd)(const SFX(or_lvl) *L, const REAL *v, int x, int k) {
  int n = L->n;
  if (x < 0 || x >= n || k < 0 || k >= n || !SFX(or_live)(L, (size_t)k * n + x)) return (REAL)0;
  return v[(size_t)k * n + x];
}

/* (A_j v)(x,k) for the 5-point stencil with face coefficients (h^2-scaled FD,
 * the stiffness block A_j of eq. full_space_optimality_system). */
static REAL SFX(or_stencil)(const SFX(or_lvl) *L, int j, const REAL *v, int x, int k) {
  int n = L->n;
  REAL kw = OR_KX(L, j, k, x), ke = OR_KX(L, j, k, x + 1);
  REAL ks = OR_KY(L, j, k, x), kn = OR_KY(L, j, k + 1, x);
  REAL diag = kw + ke + ks + kn;
  (void)n;
  return diag * SFX(or_atd)(L, v, x, k)
       - kw * SFX(or_atd)(L, v, x - 1, k) - ke * SFX(or_atd)(L, v, x + 1, k)
       - ks * SFX(or_atd)(L, v, x, k - 1) - kn * SFX(or_atd)(L, v, x, k + 1);
}

/* out = S x, block rows as in eq. (2):
 *   Y rows: C_j y_j + A_j^T p_j      (A_j is symmetric, A_j^T = A_j)
 *   U row : G u + sum_j D_j p_j
 *   P rows: A_j y_j + E_j u                                               */
static void SFX(or_apply)(const SFX(or_lvl) *L, const REAL *xv, REAL *out) {
  int n = L->n, N = L->N;
  size_t nn = (size_t)n * n;
  const REAL *U = xv + (size_t)N * nn;
  REAL *oU = out + (size_t)N * nn;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < N; ++j) {
    const REAL *Y = xv + (size_t)j * nn;
    const REAL *P = xv + (size_t)(N + 1) * nn + (size_t)j * nn;
    REAL *oY = out + (size_t)j * nn;
    REAL *oP = out + (size_t)(N + 1) * nn + (size_t)j * nn;
    for (int k = 0; k < n; ++k)
      for (int x = 0; x < n; ++x) {
        size_t i = (size_t)k * n + x;
        if (!SFX(or_live)(L, i)) { oY[i] = 0; oP[i] = 0; continue; }   /* zero rows outside */
        oY[i] = L->c[j] * Y[i] + SFX(or_stencil)(L, j, P, x, k);
        oP[i] = SFX(or_stencil)(L, j, Y, x, k) + (SFX(or_mask_e)(L, i) * L->e[j]) * U[i];
      }
  }
  for (size_t i = 0; i < nn; ++i) {
    if (!SFX(or_live)(L, i)) { oU[i] = 0; continue; }
    REAL s = L->g * U[i], mi = SFX(or_mask_d)(L, i);
    for (int j = 0; j < N; ++j) s += (mi * L->d[j]) * xv[(size_t)(N + 1) * nn + (size_t)j * nn + i];
    oU[i] = s;
  }
}

/* r = f - S x */
static void SFX(or_residual)(const SFX(or_lvl) *L, const REAL *xv, const REAL *f, REAL *r) {
  size_t nn = (size_t)L->n * L->n, len = (size_t)(2 * L->N + 1) * nn;
  SFX(or_apply)(L, xv, r);
  for (size_t i = 0; i < len; ++i) r[i] = SFX(or_live)(L, i % nn) ? f[i] - r[i] : (REAL)0;
}

/* Node solve of eq. solution_reduced_system: the (2N+1)x(2N+1) system
 * S~_i x_i = b_i of eq. reduced_matrices solved by a Schur complement on u_i.
 * bP is the right-hand side of the first (C/A^T) block row, bY that of the
 * third (A/E) block row, bU that of the control row.                       */
static void SFX(or_node_solve)(int N, const REAL *a, const REAL *c, const REAL *d,
                               const REAL *e, REAL g, const REAL *bP, REAL bU,
                               const REAL *bY, REAL *y, REAL *u, REAL *p) {
  REAL num = bU, den = g;
  for (int j = 0; j < N; ++j) {
    num += d[j] * (c[j] * bY[j] / (a[j] * a[j]) - bP[j] / a[j]);
    den += d[j] * c[j] * e[j] / (a[j] * a[j]);
  }
  REAL uu = num / den;
  for (int j = 0; j < N; ++j) {
    y[j] = (bY[j] - e[j] * uu) / a[j];
    p[j] = (bP[j] - c[j] * y[j]) / a[j];
  }
  *u = uu;
}

/* One half-sweep of the collective Gauss-Seidel smoother (eq. collective_smoothing
 * with the nodes visited by colour): every node with (x+k)%2 == colour is replaced
 * by (1-theta) x_i + theta S~_i^{-1}(b_i), where b_i holds f_i plus the couplings
 * to the (opposite-colour) neighbours.  Same-colour nodes do not couple through
 * the 5-point stencil and the diagonal blocks, so the visiting order is immaterial. */
static void SFX(or_halfsweep)(const SFX(or_lvl) *L, int colour, REAL theta,
                              REAL *xv, const REAL *f) {
  int n = L->n, N = L->N;
  size_t nn = (size_t)n * n;
  REAL *U = xv + (size_t)N * nn;
  const REAL *fU = f + (size_t)N * nn;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n; ++k) {
    REAL *a = (REAL *)malloc(sizeof(REAL) * 7 * (size_t)N);
    REAL *bP = a + N, *bY = a + 2 * N, *yn = a + 3 * N, *pn = a + 4 * N, *dm = a + 5 * N, *em = a + 6 * N;
    for (int x = 0; x < n; ++x) {
      if (((x + k) & 1) != colour) continue;
      size_t i = (size_t)k * n + x;
      if (!SFX(or_live)(L, i)) {   /* outside the domain: held at zero */
        for (int j = 0; j < N; ++j) {
          xv[(size_t)j * nn + i] = 0;
          xv[(size_t)(N + 1) * nn + (size_t)j * nn + i] = 0;
        }
        U[i] = 0;
        continue;
      }
      for (int j = 0; j < N; ++j) {
        dm[j] = SFX(or_mask_d)(L, i) * L->d[j];
        em[j] = SFX(or_mask_e)(L, i) * L->e[j];
      }
      for (int j = 0; j < N; ++j) {
        const REAL *Y = xv + (size_t)j * nn;
        const REAL *P = xv + (size_t)(N + 1) * nn + (size_t)j * nn;
        REAL kw = OR_KX(L, j, k, x), ke = OR_KX(L, j, k, x + 1);
        REAL ks = OR_KY(L, j, k, x), kn = OR_KY(L, j, k + 1, x);
        a[j] = kw + ke + ks + kn;
        bP[j] = f[(size_t)j * nn + i]
              + kw * SFX(or_atd)(L, P, x - 1, k) + ke * SFX(or_atd)(L, P, x + 1, k)
              + ks * SFX(or_atd)(L, P, x, k - 1) + kn * SFX(or_atd)(L, P, x, k + 1);
        bY[j] = f[(size_t)(N + 1) * nn + (size_t)j * nn + i]
              + kw * SFX(or_atd)(L, Y, x - 1, k) + ke * SFX(or_atd)(L, Y, x + 1, k)
              + ks * SFX(or_atd)(L, Y, x, k - 1) + kn * SFX(or_atd)(L, Y, x, k + 1);
      }
      REAL un;
      SFX(or_node_solve)(N, a, L->c, dm, em, L->g, bP, fU[i], bY, yn, &un, pn);
      for (int j = 0; j < N; ++j) {
        REAL *Y = xv + (size_t)j * nn;
        REAL *P = xv + (size_t)(N + 1) * nn + (size_t)j * nn;
        Y[i] = ((REAL)1 - theta) * Y[i] + theta * yn[j];
        P[i] = ((REAL)1 - theta) * P[i] + theta * pn[j];
      }
      U[i] = ((REAL)1 - theta) * U[i] + theta * un;
    }
    free(a);
  }
}

/* Collective damped Jacobi step, eq. collective_smoothing as printed:
 * x <- x + theta sum_i P_i S~_i^{-1} R_i (f - S x) (the smoother of the paper's
 * experiments, with theta = 1/2). */
static void SFX(or_jacobi)(const SFX(or_lvl) *L, REAL theta, REAL *xv, const REAL *f) {
  int n = L->n, N = L->N;
  size_t nn = (size_t)n * n, len = (size_t)(2 * N + 1) * nn;
  REAL *r = (REAL *)malloc(sizeof(REAL) * len);
  REAL *w = (REAL *)malloc(sizeof(REAL) * 7 * (size_t)N);
  REAL *a = w, *bP = w + N, *bY = w + 2 * N, *yn = w + 3 * N, *pn = w + 4 * N, *dm = w + 5 * N, *em = w + 6 * N;
  SFX(or_residual)(L, xv, f, r);
  for (int k = 0; k < n; ++k)
    for (int x = 0; x < n; ++x) {
      size_t i = (size_t)k * n + x;
      if (!SFX(or_live)(L, i)) {   /* outside the domain: held at zero */
        for (int j = 0; j < N; ++j) {
          xv[(size_t)j * nn + i] = 0;
          xv[(size_t)(N + 1) * nn + (size_t)j * nn + i] = 0;
        }
        xv[(size_t)N * nn + i] = 0;
        continue;
      }
      for (int j = 0; j < N; ++j) {
        dm[j] = SFX(or_mask_d)(L, i) * L->d[j];
        em[j] = SFX(or_mask_e)(L, i) * L->e[j];
        a[j] = OR_KX(L, j, k, x) + OR_KX(L, j, k, x + 1) + OR_KY(L, j, k, x) + OR_KY(L, j, k + 1, x);
        bP[j] = r[(size_t)j * nn + i];
        bY[j] = r[(size_t)(N + 1) * nn + (size_t)j * nn + i];
      }
      REAL un;
      SFX(or_node_solve)(N, a, L->c, dm, em, L->g, bP, r[(size_t)N * nn + i], bY, yn, &un, pn);
      for (int j = 0; j < N; ++j) {
        xv[(size_t)j * nn + i] += theta * yn[j];
        xv[(size_t)(N + 1) * nn + (size_t)j * nn + i] += theta * pn[j];
      }
      xv[(size_t)N * nn + i] += theta * un;
    }
  free(w);
  free(r);
}

/* Zero every field of v at the nodes outside the domain (a restricted residual
 * there is no equation of the coarse system). */
static void SFX(zero_outside)(const SFX(or_lvl) *L, REAL *v) {
  if (!L->dom) return;
  size_t nn = (size_t)L->n * L->n;
  for (int b = 0; b < 2 * L->N + 1; ++b)
    for (size_t i = 0; i < nn; ++i)
      if (!SFX(or_live)(L, i)) v[b * nn + i] = 0;
}

/* Node i of level L carries a control: a U unknown coupled to the state and
 * adjoint rows (its md or me factor nonzero, inside the domain).  The control
 * space U_h spans the basis functions of these nodes only (Section 2: a local
 * or a boundary control lives on part of the mesh), so the multigrid transfer
 * of the U block stays inside it. */
static inline int SFX(or_control)(const SFX(or_lvl) *L, size_t i) {
  return SFX(or_mask_d)(L, i) != (REAL)0 || SFX(or_mask_e)(L, i) != (REAL)0;
}

/* U block of the fine-level residual r zeroed at nodes without a control:
 * restriction of the control residual is the transpose of the control
 * prolongation below. */
static void SFX(control_residual)(const SFX(or_lvl) *L, REAL *r) {
  size_t nn = (size_t)L->n * L->n;
  REAL *U = r + (size_t)L->N * nn;
  for (size_t i = 0; i < nn; ++i)
    if (!SFX(or_control)(L, i)) U[i] = 0;
}

/* U block of the restricted residual fc (level nc) zeroed at coarse nodes
 * whose coincident fine node (level F) has no control: the coarse control
 * space is that of the fine level taken at the coarse nodes. */
static void SFX(control_coarse_rows)(const SFX(or_lvl) *F, int nc, REAL *fc) {
  REAL *U = fc + (size_t)F->N * nc * nc;
  for (int K = 0; K < nc; ++K)
    for (int X = 0; X < nc; ++X)
      if (!SFX(or_control)(F, (size_t)(2 * K + 1) * F->n + (2 * X + 1))) U[(size_t)K * nc + X] = 0;
}

/* 1D weights of bilinear interpolation: w(0)=1, w(+-1)=1/2. */
static inline REAL SFX(or_w)(int d) { return d == 0 ? (REAL)1 : (REAL)0.5; }

/* Restriction R = P^T of bilinear prolongation (full weighting with weights
 * 1, 1/2, 1/4 summing to 4), applied to every field plane; coarse node (X,K)
 * coincides with fine node (2X+1, 2K+1).                                   */
static void SFX(or_restrict)(int nf, int N, const REAL *fine, REAL *coarse) {
  int nc = (nf - 1) / 2;
  size_t nnf = (size_t)nf * nf, nnc = (size_t)nc * nc;
  for (int b = 0; b < 2 * N + 1; ++b) {
    const REAL *F = fine + b * nnf;
    REAL *C = coarse + b * nnc;
    for (int K = 0; K < nc; ++K)
      for (int X = 0; X < nc; ++X) {
        REAL s = 0;
        for (int dk = -1; dk <= 1; ++dk)
          for (int dx = -1; dx <= 1; ++dx)
            s += SFX(or_w)(dx) * SFX(or_w)(dk) * F[(size_t)(2 * K + 1 + dk) * nf + (2 * X + 1 + dx)];
        C[(size_t)K * nc + X] = s;
      }
  }
}

/* fine += P coarse, P bilinear interpolation (Alg. 1, coarse correction).
 * With the fine level Lf given, the U block is prolongated into the control
 * space only: fine nodes without a control (or_control) keep their u. */
static void SFX(or_prolong_add)(int nc, int N, const REAL *coarse, REAL *fine, const SFX(or_lvl) *Lf) {
  int nf = 2 * nc + 1;
  size_t nnf = (size_t)nf * nf, nnc = (size_t)nc * nc;
  for (int b = 0; b < 2 * N + 1; ++b) {
    const REAL *C = coarse + b * nnc;
    REAL *F = fine + b * nnf;
    for (int K = 0; K < nc; ++K)
      for (int X = 0; X < nc; ++X)
        for (int dk = -1; dk <= 1; ++dk)
          for (int dx = -1; dx <= 1; ++dx) {
            size_t i = (size_t)(2 * K + 1 + dk) * nf + (2 * X + 1 + dx);
            if (b == N && Lf && !SFX(or_control)(Lf, i)) continue;
            F[i] += SFX(or_w)(dx) * SFX(or_w)(dk) * C[(size_t)K * nc + X];
          }
  }
}
