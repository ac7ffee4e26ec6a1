"""Risk-averse OCPUU with the smoothed CVaR (Section 6, eq. OCP), solved by the
nonlinear preconditioned Newton method of Algorithm 3.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Vectors use the paper's
layout of eq. (2): x = [y_1..y_N | u | p_1..p_N], each block n x n; t is a
separate scalar.

Scaling.  As for the linear-quadratic problems of this package, the adjoint is
carried rescaled by the sample weights (p~_j = zeta_j p_j) and the Y rows are
those of the paper times zeta_j; M = h^2 I is the lumped mass.  With
z_j = M (y_j - y_d) (zero outside the domain) and
Q_j = (1/2) (y_j - y_d)^T M (y_j - y_d) - t, the residual of
eq. discretized_nonlinearsystem reads

    F_Y,j = c_j (y_j - y_d) + A_j^T p~_j,   c_j = zeta_j g'(Q_j) h^2 / (1 - lambda)
    F_U   = nu M u - M sum_j p~_j
    F_P,j = A_j y_j - M (u + f)
    F_4   = 1 - sum_j zeta_j g'(Q_j) / (1 - lambda)

i.e. F_1 = S(c) x - b(c): the linear-quadratic operator with per-sample
C_j = c_j I (c_j >= 0) and right-hand side b(c) = [c_j y_d | f_U | f_P].  The
Jacobian blocks of eq. optmality_systeMmoothed_discretized in these rows, with
w_j = zeta_j g''(Q_j) / (1 - lambda):

    J_11 = S(c) + diag_j(w_j z_j z_j^T) in the Y-Y blocks
    J_12 = [-w_j z_j | 0 | 0],  J_21 = [-w_j z_j^T | 0 | 0],  J_22 = sum_j w_j.

Linear solves with J_11 (the paper solves them with the collective multigrid,
as a V-cycle iteration and inside GMRES): the multigrid hierarchy is the one of
S(c) (the pointwise-relaxable part; coarse levels 4^l c_j), and the rank-one
terms enter the fine-level operator only:

  * "gmres": GMRES(30) right-preconditioned by one V-cycle for S(c) from zero,
    its Arnoldi products with J_11;
  * "vcycle": the stationary iteration x <- x + V(b - J_11 x), one V-cycle for
    S(c) from zero on the exact residual of J_11.

Both stop at ||b - J_11 x|| <= 1e-9 ||b|| (80 iterations at most for GMRES,
as in the paper; 300 for the V-cycle iteration).

Readings (the paper leaves them open): the smoothing function's middle branch is
g(x) = s^3/eps^2 - s^4/(2 eps^3) with s = x + eps/2 (the printed branch has a
typo; this is the C^2 piece that joins 0 and x); t^0 = 0; the Newton iterates
for h(t) start from the current x; the inner Newton stops by the printed rule
max(||F_1(x^k)|| / ||F_1(x^0)||, ||F_1(x^k)||) <= 1e-8 with x^0 the start of that
inner iteration; an evaluation that cannot meet the relative part (a warm start
whose ||F_1(x^0)|| is within 1e8 of the rounding floor) runs to the iteration
cap or stalls (below); the paper names Newton's method for h(t) without its
globalization, and full steps cycle on its Monte Carlo problems (705 nodes,
N = 100: ||F_1|| stays at 3e-3..6e-3 for 50 steps), so each step backtracks on
||F_1|| and the iteration ends when no halving decreases it (the rounding
floor) (full steps: ``inner_backtrack=False``; the rule with min:
``inner_rule="min"``; neither is a default);
the split step solves F_2(x; t) = 0 by bisection (F_2 is nondecreasing in t)
and then recomputes x = h(t) at the new t, since F(t) = F_2(h(t), t) is what the
next test reads;
the line search of the outer Newton uses sigma = 1e-4, rho = 1/2.
"""
from __future__ import annotations

import numpy as np

from .oracle import Oracle


def g_eps(x, eps):
    """The C^2 smoothing of max(0, x) (eq. smoothapproximation)."""
    x = np.asarray(x, dtype=np.float64)
    s = np.clip(x + 0.5 * eps, 0.0, eps)            # the middle branch's variable, on its interval
    mid = s ** 3 / eps ** 2 - s ** 4 / (2 * eps ** 3)
    return np.where(x <= -0.5 * eps, 0.0, np.where(x >= 0.5 * eps, x, mid))


def dg_eps(x, eps):
    x = np.asarray(x, dtype=np.float64)
    s = np.clip(x + 0.5 * eps, 0.0, eps)
    mid = 3 * s ** 2 / eps ** 2 - 2 * s ** 3 / eps ** 3
    return np.where(x <= -0.5 * eps, 0.0, np.where(x >= 0.5 * eps, 1.0, mid))


def ddg_eps(x, eps):
    x = np.asarray(x, dtype=np.float64)
    s = np.clip(x + 0.5 * eps, 0.0, eps)
    mid = 6 * s / eps ** 2 - 6 * s ** 2 / eps ** 3
    return np.where((x <= -0.5 * eps) | (x >= 0.5 * eps), 0.0, mid)


class Cvar:
    """The smoothed risk-averse problem on a linear-quadratic problem's data
    (faces, weights zeta_j = c_j / h^2, y_d, f, nu, domain)."""

    def __init__(self, prob, lam: float, eps: float, smoother: str = "jacobi", theta: float = 0.5):
        if not (0 <= lam < 1) or not eps > 0:
            raise ValueError("need 0 <= lambda < 1 and eps > 0")
        self.p, self.lam, self.eps = prob, lam, eps
        self.n, self.N = prob.n, prob.N
        self.nn = prob.n * prob.n
        self.mass = -float(prob.d[0])                      # D_j = -M
        self.zeta = np.asarray(prob.c, dtype=np.float64) / self.mass
        dom = getattr(prob, "domain", None)
        self.live = np.ones(self.nn) if dom is None else np.asarray(dom, dtype=np.float64).reshape(self.nn)
        self.yd = np.asarray(prob.yd, dtype=np.float64).reshape(self.nn) * self.live
        self.o = Oracle(prob, smoother=smoother, theta=theta)

    # --- pieces of F and J -------------------------------------------------
    def blocks(self, x):
        N, nn = self.N, self.nn
        return x[:N * nn].reshape(N, nn), x[N * nn:(N + 1) * nn], x[(N + 1) * nn:].reshape(N, nn)

    def z_q(self, x):
        """z_j = M (y_j - y_d) on the domain and q_j = Q_j + t."""
        Y = self.blocks(x)[0]
        z = self.mass * (Y - self.yd[None]) * self.live[None]
        return z, 0.5 * np.sum(z * z, axis=1) / self.mass

    def c_of(self, q, t):
        return self.zeta * dg_eps(q - t, self.eps) * self.mass / (1 - self.lam)

    def w_of(self, q, t):
        return self.zeta * ddg_eps(q - t, self.eps) / (1 - self.lam)

    def F4(self, q, t):
        return 1.0 - np.sum(self.zeta * dg_eps(q - t, self.eps)) / (1 - self.lam)

    def rhs(self, c):
        p = self.p
        fY = c[:, None] * self.yd[None]
        return np.concatenate([fY.ravel(), p.fU.ravel(), p.fP.ravel()])

    def F1(self, x, t):
        """F_1(x; t); also sets the oracle's C_j = c_j(x, t) I."""
        _, q = self.z_q(x)
        c = self.c_of(q, t)
        self.o.set_sample_c(c)
        return -self.o.residual(x, self.rhs(c))

    def J11(self, v, w, z):
        out = self.o.apply(v)
        N, nn = self.N, self.nn
        V = v[:N * nn].reshape(N, nn)
        out[:N * nn] += (w[:, None] * z * np.sum(z * V, axis=1)[:, None]).ravel()
        return out

    # --- linear solves with J_11 ------------------------------------------
    def solve(self, b, w, z, method: str, tol: float = 1e-9):
        bn = np.linalg.norm(b)
        if bn == 0.0:
            return np.zeros_like(b), 0
        if method == "vcycle":
            x = np.zeros_like(b)
            for k in range(301):
                r = b - self.J11(x, w, z)
                if np.linalg.norm(r) <= tol * bn or k == 300:
                    return x, k
                x = x + self.o.vcycle(np.zeros_like(b), r, 1)
        return self._gmres(b, w, z, tol, 30, 80)

    def _gmres(self, b, w, z, tol, m, maxit):
        """GMRES(m), right preconditioner one V-cycle for S(c) from zero,
        modified Gram-Schmidt; x0 = 0."""
        bn = np.linalg.norm(b)
        x = np.zeros_like(b)
        its = 0
        while True:
            r = b - self.J11(x, w, z)
            beta = np.linalg.norm(r)
            if beta <= tol * bn or its >= maxit:
                return x, its
            V = [r / beta]
            Zs, H = [], np.zeros((m + 1, m))
            g = np.zeros(m + 1)
            g[0] = beta
            k = 0
            while k < m and its < maxit:
                zk = self.o.vcycle(np.zeros_like(b), V[k], 1)
                Zs.append(zk)
                v = self.J11(zk, w, z)
                for i in range(k + 1):
                    H[i, k] = V[i] @ v
                    v = v - H[i, k] * V[i]
                H[k + 1, k] = np.linalg.norm(v)
                its += 1
                k += 1
                y, res = _lsq(H[:k + 1, :k], g[:k + 1])
                if res <= tol * bn or H[k, k - 1] == 0.0:
                    break
                V.append(v / H[k, k - 1])
            x = x + np.array(Zs).T @ y

    # --- the two Newton iterations ----------------------------------------
    def inner(self, x, t, method, tol=1e-8, maxit=50, lin=None, rule="max", backtrack=True, hist=None):
        """h(t): Newton on F_1(.; t) = 0 from x.

        rule="max" (Section 6, the stopping rules stated with the risk-averse
        table): stop once max(||F_1(x^k)|| / ||F_1(x^0)||, ||F_1(x^k)||) <= tol,
        i.e. both the relative and the absolute residual are small; rule="min"
        (a named variant, not the paper's) stops once either part is.
        backtrack=True halves each step (1, 1/2, ..., at most 30 halvings)
        until ||F_1(x + a dx)|| <= (1 - 1e-4 a) ||F_1(x)||: Algorithm 3 names
        Newton's method for h without its globalization, and full steps
        (backtrack=False) cycle on the paper's Monte Carlo problems.  When no
        halving decreases ||F_1|| although the absolute part is met
        (||F_1|| <= tol: the relative part is out of reach at the rounding
        floor) the iteration ends there without the step ("stalled"); with a
        larger residual the last halving is taken.  hist (a list) receives
        ||F_1|| at every iterate.  Returns (x, Newton steps taken, stalled)."""
        if rule not in ("max", "min"):
            raise ValueError("rule must be 'max' or 'min'")
        stop = max if rule == "max" else min
        x = np.array(x, dtype=np.float64)
        F = self.F1(x, t)
        fn = f0 = np.linalg.norm(F)
        if hist is not None:
            hist.append(fn)
        k = 0
        while k < maxit:
            if fn == 0.0 or stop(fn / f0, fn) <= tol:
                break
            z, q = self.z_q(x)
            dx, its = self.solve(-F, self.w_of(q, t), z, method)
            if lin is not None:
                lin.append(its)
            a = 1.0
            ok = not backtrack
            for ls in range(31 if backtrack else 1):
                xt = x + a * dx
                Ft = self.F1(xt, t)
                ft = np.linalg.norm(Ft)
                if not backtrack or ft <= (1.0 - 1e-4 * a) * fn:
                    ok = True
                    break
                if ls < 30:
                    a *= 0.5
            if not ok and fn <= tol:                       # no decrease at the floor
                self.F1(x, t)                              # C_j back at x
                return x, k, True
            x, F, fn = xt, Ft, ft
            if hist is not None:
                hist.append(fn)
            k += 1
        return x, k, False

    def split_t(self, q):
        """The root of F_2(x; t) = 0 for fixed x (bisection)."""
        lo, hi = float(q.min()) - self.eps, float(q.max()) + self.eps
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid == lo or mid == hi:
                break
            if self.F4(q, mid) < 0.0:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi)

    def run(self, method: str = "gmres", t0: float = 0.0, tol: float = 1e-6, maxit: int = 50,
            sigma: float = 1e-4, rho: float = 0.5, max_ls: int = 30, x0=None, inner_tol: float = 1e-8,
            inner_maxit: int = 50, inner_rule: str = "max", inner_backtrack: bool = True):
        """Algorithm 3.  Returns t, x, u, the outer and inner Newton counts, the
        Newton count of every evaluation of h (``inner_counts``; an entry equal
        to inner_maxit is an evaluation that ended at the cap) and whether it
        stalled at the rounding floor (``inner_stalled``), the
        linear-solver iterations of every solve and |F(t^k)| per iterate."""
        lin, counts = [], []
        t = float(t0)
        x = np.zeros((2 * self.N + 1) * self.nn) if x0 is None else np.array(x0, dtype=np.float64)
        base_inner = self.inner

        stalled = []

        def inner(x, t, method, lin=None):
            xx, kk, st = base_inner(x, t, method, tol=inner_tol, maxit=inner_maxit, lin=lin, rule=inner_rule,
                                    backtrack=inner_backtrack)
            counts.append(kk)
            stalled.append(st)
            return xx, kk
        x, inner_total = inner(x, t, method, lin=lin)
        hist, k, converged = [], 0, False
        while True:
            z, q = self.z_q(x)
            Ft = self.F4(q, t)
            hist.append(abs(Ft))
            if abs(Ft) <= tol:
                converged = True
                break
            if k >= maxit:
                break
            w = self.w_of(q, t)
            if not np.any(w != 0.0):                       # eq. condition: split step
                x, kk = inner(x, t, method, lin=lin)
                inner_total += kk
                t = self.split_t(self.z_q(x)[1])
                # F(t) = F_2(h(t), t): the next test needs h at the new t
                x, kk = inner(x, t, method, lin=lin)
                inner_total += kk
            else:
                self.F1(x, t)                              # S(c) at (x^k, t^k)
                rhs = np.zeros_like(x)
                rhs[:self.N * self.nn] = (-w[:, None] * z).ravel()
                xi, its = self.solve(rhs, w, z, method)
                lin.append(its)
                Xi = xi[:self.N * self.nn].reshape(self.N, self.nn)
                Fp = np.sum(w) + np.sum(w * np.sum(z * Xi, axis=1))
                d = -Ft / Fp
                gamma = 1.0
                for ls in range(max_ls + 1):
                    xt, kk = inner(x, t + gamma * d, method, lin=lin)
                    inner_total += kk
                    Fn = self.F4(self.z_q(xt)[1], t + gamma * d)
                    if abs(Fn) - abs(Ft) <= -sigma * abs(Ft):
                        break
                    if ls < max_ls:
                        gamma *= rho
                t, x = t + gamma * d, xt
            k += 1
        u = self.blocks(x)[1].copy()
        return dict(t=t, x=x, u=u, outer=k, inner_total=inner_total, inner_counts=counts,
                    inner_capped=sum(1 for c in counts if c >= inner_maxit), inner_stalled=stalled,
                    linear=lin, F=hist, converged=converged)

    def objective(self, y_of_u, u, t):
        """t + E[g(Q)] / (1 - lambda) + nu/2 u^T M u for states y_of_u(u) (N, nn)."""
        Y = y_of_u(u)
        z = self.mass * (Y - self.yd[None]) * self.live[None]
        q = 0.5 * np.sum(z * z, axis=1) / self.mass
        return (t + np.sum(self.zeta * g_eps(q - t, self.eps)) / (1 - self.lam)
                + 0.5 * self.p.nu * self.mass * np.sum(u * u))


def _lsq(H, g):
    """min ||g - H y|| by dense least squares; returns y and the residual norm."""
    y, *_ = np.linalg.lstsq(H, g, rcond=None)
    return y, float(np.linalg.norm(g - H @ y))
