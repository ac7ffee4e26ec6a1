"""Globalized semismooth Newton method for the OCPUU with an L^1 penalty and box
constraints on the control (Section 5, eq. l1_OCP, Algorithm 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Vectors use the paper's
layout of eq. (2): x = [y_1..y_N | u | p_1..p_N], each block n x n.

Scaling.  The problems of this package carry the adjoint rescaled by the
sample weights, p~_j = zeta_j p_j (C_j = zeta_j M, D_j = E_j = -M, M = h^2 I),
so the expectation of eq. nonlinear_optimality_condition's discrete form is
E[p] = sum_j zeta_j p_j = sum_j p~_j.  The Newton system
eq. full_space_optimality_systeMemismooth2 in the same unknowns
(H^k = chi / nu, chi the indicator of I+ u I-):

    C_j dy_j + A_j dp~_j = 0
    M du - (1/nu) sum_j chi M dp~_j = -M F(u)
    A_j dy_j + E_j du = 0

i.e. the linear-quadratic operator with its U row divided by nu (G = M,
D_j / nu; ``newton_problem``) and the node entries of D_j multiplied by chi_i
(node factor md = chi, me = 1).  The printed right side of the U row omits
the mass matrix; the Galerkin form of G(u) du = -F(u) carries it (-M F),
which is what is used here.  Keeping the printed row scale (rather than the
linear-quadratic system's nu M) matters for the stopping test: the right side
lives in the U row alone, and with that row scaled by nu a relative residual
of 1e-11 lies below what FP64 rounding in the Y and P rows allows.

Line search (Algorithm 2, the inner while): the merit is
phi(u) = sqrt(F(u)^T M F(u)) = h ||F(u)||; a step gamma is accepted once
phi(u + gamma du) - phi(u) <= -sigma phi(u).  y and p are affine in u and the
Newton increments solve the linearized state and adjoint equations, so
E[p](u + gamma du) = E[p](u) + gamma E[dp]: no extra solves.
sigma and rho are not printed; sigma = 1e-4, rho = 1/2 are used.

Coarse levels of the multigrid inner solves carry the active set by full
weighting (the lumped diagonal of the Galerkin product R diag(chi) P, the
paper's coarse operators being Galerkin ones): injection keeps only every
other node's indicator and the V-cycle then needs three to five times as many
cycles per Newton step.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .oracle import Oracle


# ---------------------------------------------------------------- pointwise maps
def F_map(u, w, nu, beta, a, b):
    """F(u) of the discrete optimality condition (Section 5), componentwise in
    w = E[p], in the printed max/min form."""
    u = np.asarray(u, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    s = (np.maximum(0.0, w - beta) + np.minimum(0.0, w + beta)
         - np.maximum(0.0, w - beta - nu * b) - np.minimum(0.0, w + beta - nu * a))
    return u - s / nu


def active_set(w, nu, beta, a, b):
    """Indicator of I+ u I- (eq. activesets) as float64 0/1."""
    w = np.asarray(w, dtype=np.float64)
    ip = (w - beta >= 0.0) & (w - beta <= nu * b)
    im = (w + beta >= nu * a) & (w + beta <= 0.0)
    return (ip | im).astype(np.float64)


def merit(F, h):
    """phi = sqrt(F^T M F), M = h^2 I."""
    F = np.asarray(F, dtype=np.float64)
    return float(h * np.sqrt(np.dot(F, F)))


def expected_p(x, n, N):
    """E[p] = sum_j p~_j from a vector in the paper's layout."""
    nn = n * n
    return np.asarray(x[(N + 1) * nn:], dtype=np.float64).reshape(N, nn).sum(axis=0)


def newton_problem(prob):
    """The problem data of the Newton system: the U row of the linear-quadratic
    system divided by nu (G = M, D_j / nu); the rest unchanged."""
    return dataclasses.replace(prob, g=prob.g / prob.nu, d=np.asarray(prob.d) / prob.nu)


# ---------------------------------------------------------------- sparse blocks
def _on_domain(prob, M, fields):
    """M restricted to the problem's domain: rows and columns of the unknowns of
    nodes outside become identity ones (M unchanged without a domain).  fields:
    how many n x n planes the matrix acts on."""
    if getattr(prob, "domain", None) is None:
        return M
    live = np.tile(np.asarray(prob.domain, dtype=np.float64).ravel(), fields)
    D = sp.diags(live)
    return (D @ M @ D + sp.diags(1.0 - live)).tocsc()


def stiffness(prob, j):
    """A_j: the h^2-scaled 5-point stencil of sample j from its face coefficients
    (on the problem's domain: the Dirichlet problem there, identity rows outside)."""
    return _on_domain(prob, _stiffness_square(prob, j), 1)


def _stiffness_square(prob, j):
    n = prob.n
    kx, ky = prob.kx[j], prob.ky[j]
    rows, cols, vals = [], [], []
    for k in range(n):
        for x in range(n):
            i = k * n + x
            kw, ke, ks, kn = kx[k, x], kx[k, x + 1], ky[k, x], ky[k + 1, x]
            rows.append(i); cols.append(i); vals.append(kw + ke + ks + kn)
            for (xx, kk, c) in ((x - 1, k, kw), (x + 1, k, ke), (x, k - 1, ks), (x, k + 1, kn)):
                if 0 <= xx < n and 0 <= kk < n:
                    rows.append(i); cols.append(kk * n + xx); vals.append(-c)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n * n, n * n))


def assemble(prob, md=None, me=None):
    """Sparse S of eq. (2) with node factors md on D_j and me on E_j (None: 1)."""
    n, N = prob.n, prob.N
    nn = n * n
    md = np.ones(nn) if md is None else np.asarray(md, dtype=np.float64).ravel()
    me = np.ones(nn) if me is None else np.asarray(me, dtype=np.float64).ravel()
    I = sp.identity(nn, format="csr")
    blocks = [[None] * (2 * N + 1) for _ in range(2 * N + 1)]
    for j in range(N):
        A = stiffness(prob, j)
        blocks[j][j] = prob.c[j] * I
        blocks[j][N + 1 + j] = A.T
        blocks[N][N + 1 + j] = sp.diags(md * prob.d[j])
        blocks[N + 1 + j][j] = A
        blocks[N + 1 + j][N] = sp.diags(me * prob.e[j])
    blocks[N][N] = prob.g * I
    return _on_domain(prob, sp.bmat(blocks, format="csc"), 2 * N + 1)


def initial_state(prob, u0):
    """Algorithm 2, first step: y_j = A_j^{-1}(f_P,j - E_j u0) and
    p~_j = A_j^{-T}(f_Y,j - C_j y_j) (with the package's scaling these are
    A_j^{-1} M (f + u0) and zeta_j A_j^{-T} M (y_d - y_j))."""
    n, N = prob.n, prob.N
    nn = n * n
    u0 = np.asarray(u0, dtype=np.float64).ravel()
    if getattr(prob, "domain", None) is not None:
        u0 = u0 * np.asarray(prob.domain).ravel()     # no control outside the domain
    x = np.zeros((2 * N + 1) * nn)
    x[N * nn:(N + 1) * nn] = u0
    for j in range(N):
        lu = spla.splu(stiffness(prob, j).tocsc())
        live = 1.0 if getattr(prob, "domain", None) is None else np.asarray(prob.domain).ravel()
        y = lu.solve(live * (prob.fP[j].ravel() - prob.e[j] * u0))
        p = lu.solve(live * (prob.fY[j].ravel() - prob.c[j] * y), trans="T")
        x[j * nn:(j + 1) * nn] = y
        x[(N + 1 + j) * nn:(N + 2 + j) * nn] = p
    return x


# ---------------------------------------------------------------- Algorithm 2
def ssn_solve(prob, beta, a, b, *, u0=None, tol=1e-9, linear="direct", inner_tol=1e-11,
              sigma=1e-4, rho=0.5, maxit=100, smoother="gs", theta=1.0, gmres_m=30,
              inner_maxit=500, max_backtracks=60, keep_steps=False):
    """Solve F(u) = 0 by Algorithm 2.

    linear: how each Newton system is solved: "direct" (sparse LU of the
    assembled S), "vcycle" (stationary V(2,2) of the oracle to inner_tol,
    relative residual) or "gmres" (GMRES(gmres_m) with the V-cycle as right
    preconditioner).  Returns a dict with x (paper layout), u, w = E[p],
    iterations, phi (merit history, one entry per iterate), gammas, inner
    (iterations of each linear solve) and chi (final active-set indicator);
    with keep_steps, also steps = [(u_k, du_k)] of every Newton iteration.
    """
    if getattr(prob, "ctrl", None) is not None:
        raise ValueError("the semismooth Newton method is set up for control everywhere")
    n, N = prob.n, prob.N
    nn = n * n
    h = 1.0 / (n + 1)
    nu = prob.nu
    if not (nu > 0 and beta >= 0 and a < 0 < b):
        raise ValueError("need nu > 0, beta >= 0 and a < 0 < b")
    u0 = np.zeros(nn) if u0 is None else np.asarray(u0, dtype=np.float64).ravel()
    x = initial_state(prob, u0)
    pn = newton_problem(prob)
    orc = None
    if linear in ("vcycle", "gmres"):
        orc = Oracle(pn, smoother=smoother, theta=theta)
    elif linear != "direct":
        raise ValueError("linear must be 'direct', 'vcycle' or 'gmres'")
    U = slice(N * nn, (N + 1) * nn)
    w = expected_p(x, n, N)
    Fv = F_map(x[U], w, nu, beta, a, b)
    chi = active_set(w, nu, beta, a, b)
    phi = merit(Fv, h)
    hist, gammas, inner, steps = [phi], [], [], []
    k = 0
    while phi > tol and k < maxit:
        r = np.zeros_like(x)
        r[U] = -pn.g * Fv
        if linear == "direct":
            dx = spla.spsolve(assemble(pn, md=chi), r)
            inner.append(1)
        else:
            orc.set_masks(chi.reshape(n, n), None, coarsen="full")
            if linear == "vcycle":
                dx, its, _ = orc.solve_vcycle(r, tol=inner_tol, maxit=inner_maxit)
            else:
                dx, its, _ = orc.gmres(r, m=gmres_m, tol=inner_tol, maxit=inner_maxit)
            if its < 0:
                raise RuntimeError("inner linear solve did not converge")
            inner.append(int(its))
        dw = expected_p(dx, n, N)
        if keep_steps:
            steps.append((x[U].copy(), dx[U].copy()))
        gamma = 1.0
        for _ in range(max_backtracks):
            trial = merit(F_map(x[U] + gamma * dx[U], w + gamma * dw, nu, beta, a, b), h)
            if trial - phi <= -sigma * phi:
                break
            gamma *= rho
        else:
            raise RuntimeError("line search found no decrease")
        x = x + gamma * dx
        w = expected_p(x, n, N)
        Fv = F_map(x[U], w, nu, beta, a, b)
        chi = active_set(w, nu, beta, a, b)
        phi = merit(Fv, h)
        hist.append(phi)
        gammas.append(gamma)
        k += 1
    return dict(x=x, u=x[U].copy(), w=w, iterations=k, phi=hist, gammas=gammas, inner=inner,
                chi=chi, converged=phi <= tol, steps=steps)
