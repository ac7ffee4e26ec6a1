"""Pins of the smoothed-CVaR oracle (Section 6, Algorithm 3) against facts
independent of its code: the smoothing function's joins and derivatives, the
Rockafellar-Uryasev identity (the minimum over t is the mean of the upper tail
of a discrete distribution), the Jacobian blocks against finite differences of
the residual, and the computed (u, t) as a stationary point of the objective
evaluated with sparse direct state solves assembled here."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from paper_2302_13680_amd import inputs

cv = pytest.importorskip("oracle.cvar")


def test_smoothing_function():
    eps = 0.2
    g, dg, ddg = cv.g_eps, cv.dg_eps, cv.ddg_eps
    a, b = -eps / 2, eps / 2
    d = 1e-9
    for f in (g, dg, ddg):                                 # C^2 joins (jumps of order d / eps^2)
        assert abs(f(a - d, eps) - f(a + d, eps)) < 1e-6
        assert abs(f(b - d, eps) - f(b + d, eps)) < 1e-6
    assert abs(g(0.0, eps) - 3 * eps / 32) < 1e-15
    x = np.linspace(-0.3, 0.3, 601)
    assert np.all(g(x, eps) >= np.maximum(x, 0) - 1e-15)
    assert np.all(g(x, eps) - np.maximum(x, 0) <= 3 * eps / 32 + 1e-15)
    assert np.all(np.diff(dg(x, eps)) >= -1e-15) and dg(x, eps).min() == 0 and dg(x, eps).max() == 1
    h = 1e-6
    np.testing.assert_allclose((g(x + h, eps) - g(x - h, eps)) / (2 * h), dg(x, eps), atol=1e-8)
    # g'' has kinks at the joins, where the central difference is first order
    np.testing.assert_allclose((dg(x + h, eps) - dg(x - h, eps)) / (2 * h), ddg(x, eps), atol=1e-4)


def test_split_root_gives_the_upper_tail_mean():
    """min_t t + E[g(X - t)] / (1 - lambda) -> mean of the top (1 - lambda) N values
    (Rockafellar-Uryasev) as eps -> 0; the root of F_2 attains it."""
    rng = np.random.default_rng(0)
    X = rng.uniform(0, 1, 40)
    lam, eps = 0.9, 1e-6

    class P:   # the pieces of Cvar used by split_t / F4
        pass
    c = P()
    c.zeta, c.lam, c.eps = np.full(40, 1 / 40), lam, eps
    c.F4 = lambda q, t: cv.Cvar.F4(c, q, t)
    t = cv.Cvar.split_t(c, X)
    val = t + np.sum(c.zeta * cv.g_eps(X - t, eps)) / (1 - lam)
    assert abs(val - np.sort(X)[-4:].mean()) < 1e-5
    assert abs(c.F4(X, t)) < 1e-9 or np.sort(X)[-5] + eps / 2 <= t <= np.sort(X)[-4] - eps / 2


def _problem(n=15, N=8, seed=3):
    return inputs.make_problem(n, N, 1e-3, M=3, sigma=0.5, seed=seed, domain="lshape",
                               field="gaussian", corr_len2=0.5)


def _stiffness(p, j):
    n = p.n
    rows, cols, vals = [], [], []
    for k in range(n):
        for x in range(n):
            i = k * n + x
            kw, ke, ks, kn = p.kx[j, k, x], p.kx[j, k, x + 1], p.ky[j, k, x], p.ky[j, k + 1, x]
            rows.append(i); cols.append(i); vals.append(kw + ke + ks + kn)
            for c, v in ((i - 1, -kw) if x > 0 else (None, 0), (i + 1, -ke) if x < n - 1 else (None, 0),
                         (i - n, -ks) if k > 0 else (None, 0), (i + n, -kn) if k < n - 1 else (None, 0)):
                if c is not None:
                    rows.append(i); cols.append(c); vals.append(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n * n, n * n))


def test_jacobian_blocks_match_finite_differences():
    p = _problem()
    c = cv.Cvar(p, 0.5, 0.5)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2 * p.N + 1) * p.n * p.n) * 0.3
    x[:p.N * c.nn] *= np.tile(c.live, p.N)
    z, q = c.z_q(x)
    t = float(np.median(q))                       # several samples inside the smoothing band
    w = c.w_of(q, t)
    assert np.count_nonzero(w) >= 2
    v = rng.standard_normal(x.size) * np.concatenate([np.tile(c.live, p.N), c.live, np.tile(c.live, p.N)])
    d = 1e-6
    c.F1(x, t)
    Jv = c.J11(v, w, z)
    fd = (c.F1(x + d * v, t) - c.F1(x - d * v, t)) / (2 * d)
    assert np.linalg.norm(Jv - fd) <= 1e-6 * np.linalg.norm(fd)
    J12 = np.zeros_like(x)
    J12[:p.N * c.nn] = (-w[:, None] * z).ravel()
    fdt = (c.F1(x, t + d) - c.F1(x, t - d)) / (2 * d)
    assert np.linalg.norm(J12 - fdt) <= 1e-6 * np.linalg.norm(fdt)
    J21v = -np.sum(w * np.sum(z * v[:p.N * c.nn].reshape(p.N, -1), axis=1))
    fd21 = (c.F4(c.z_q(x + d * v)[1], t) - c.F4(c.z_q(x - d * v)[1], t)) / (2 * d)
    assert abs(J21v - fd21) <= 1e-6 * abs(fd21)
    fd22 = (c.F4(q, t + d) - c.F4(q, t - d)) / (2 * d)
    assert abs(np.sum(w) - fd22) <= 1e-6 * abs(fd22)


@pytest.mark.parametrize("method", ["gmres", "vcycle"])
def test_solution_is_a_stationary_point_of_the_objective(method):
    p = _problem()
    lam, eps = 0.5, 0.05
    c = cv.Cvar(p, lam, eps)
    res = c.run(method)
    assert res["converged"] and res["outer"] >= 1
    n, N, nn = p.n, p.N, p.n * p.n
    live = c.live.astype(bool)
    A = [_stiffness(p, j)[live][:, live].tocsc() for j in range(N)]
    lu = [spla.splu(a) for a in A]
    fP = p.fP.reshape(N, nn)

    def states(u):
        Y = np.zeros((N, nn))
        for j in range(N):
            Y[j, live] = lu[j].solve(c.mass * u[live] + fP[j, live])
        return Y

    u, t = res["u"], res["t"]
    rng = np.random.default_rng(2)
    J = lambda uu, tt: c.objective(states, uu, tt)
    h = 1e-5
    scale = 0.0
    for _ in range(3):
        dvec = rng.standard_normal(nn) * c.live
        dvec /= np.linalg.norm(dvec)
        g0 = (J(h * dvec, 0.0) - J(-h * dvec, 0.0)) / (2 * h)      # away from the optimum
        g1 = (J(u + h * dvec, t) - J(u - h * dvec, t)) / (2 * h)
        scale = max(scale, abs(g0))
        assert abs(g1) <= 1e-5 * abs(g0) + 1e-12, (g0, g1)
    gt = (J(u, t + h) - J(u, t - h)) / (2 * h)
    assert abs(gt) <= 1e-5
    # the iterate's state is the state of its control
    np.testing.assert_allclose(c.blocks(res["x"])[0][:, live], states(u)[:, live], rtol=0, atol=1e-8)


def test_both_linear_solvers_agree():
    p = _problem()
    a = cv.Cvar(p, 0.5, 0.05).run("gmres")
    b = cv.Cvar(p, 0.5, 0.05).run("vcycle")
    assert a["outer"] == b["outer"]
    assert abs(a["t"] - b["t"]) <= 1e-7 * max(1.0, abs(a["t"]))
    assert np.abs(a["u"] - b["u"]).max() <= 1e-6 * np.abs(a["u"]).max()


def _quadratic_trace(c, t):
    """||F_1|| along the inner Newton iteration at t from a point near h(t)."""
    x0 = np.zeros(c.o.vlen())
    xh, _, _ = c.inner(x0, t, "gmres", tol=1e-14, maxit=30)     # close to h(t)
    hist = []
    c.inner(xh, t + 5e-2, "gmres", tol=1e-14, maxit=8, hist=hist)
    return hist


def test_inner_newton_converges_quadratically():
    """Newton's method for h(t) (Algorithm 3, the inner iteration) with the exact
    Jacobian J_11 = S(c) + w_j z_j z_j^T contracts quadratically near the root:
    ||F_1(x^{k+1})|| <= K ||F_1(x^k)||^2 until the rounding floor, with
    several samples inside the smoothing band (w_j != 0).  A Jacobian missing its
    rank-one terms (a plausible mistake) only contracts linearly and fails."""
    p = _problem()
    c = cv.Cvar(p, 0.5, 0.5)
    z, q = c.z_q(np.zeros(c.o.vlen()))
    t = float(np.median(q))
    assert np.count_nonzero(c.w_of(q, t)) >= 2

    def check(hist):
        steps = [(a, b) for a, b in zip(hist, hist[1:]) if b > 1e-14]   # above the floor (~2e-15)
        assert len(steps) >= 3, hist
        for a, b in steps:
            assert b <= 1e2 * a * a, (a, b, hist)      # quadratic; the exact Jacobian gives K ~ 30
        assert hist[-1] <= 1e-12, hist
    check(_quadratic_trace(c, t))

    class NoRankOne(cv.Cvar):
        def J11(self, v, w, z):
            return self.o.apply(v)
    bad = NoRankOne(p, 0.5, 0.5)
    with pytest.raises(AssertionError):
        check(_quadratic_trace(bad, t))


def test_inner_stopping_rules():
    """The printed rule (max of relative and absolute residual) stops later than
    the min variant and never before both parts are below the tolerance; an
    evaluation whose start sits within 1/tol of the rounding floor runs to the
    cap under the printed rule."""
    p = _problem()
    c = cv.Cvar(p, 0.5, 0.05)
    x0 = np.zeros(c.o.vlen())
    for rule in ("max", "min"):
        hist = []
        x, k, _ = c.inner(x0, 0.0, "gmres", rule=rule, hist=hist)
        assert k == len(hist) - 1
        rel, ab = hist[-1] / hist[0], hist[-1]
        if rule == "max":
            assert max(rel, ab) <= 1e-8 and k < 50
            kmax = k
        else:
            assert min(rel, ab) <= 1e-8 and k <= kmax
    # from h(0) itself: ||F_1(x^0)|| is at the floor, the relative part cannot be
    # met: full steps run to the cap, the backtracking ends at the floor
    hist = []
    _, k, st = c.inner(x, 0.0, "gmres", rule="max", maxit=4, hist=hist, backtrack=False)
    assert k == 4 and not st and max(hist) < 1e-10
    _, k, st = c.inner(x, 0.0, "gmres", rule="max", maxit=4)
    assert st or k == 4
    _, k, _ = c.inner(x, 0.0, "gmres", rule="min", maxit=4)
    assert k == 0


def test_named_variants_reach_the_same_solution():
    """The printed rule with backtracking (the default), the min rule and full
    Newton steps (named options) find the same (u, t) on a problem where full
    steps converge; the min rule stops no later than the printed one."""
    p = _problem()
    a = cv.Cvar(p, 0.5, 0.05).run("gmres")
    for kw in (dict(inner_rule="min"), dict(inner_backtrack=False)):
        b = cv.Cvar(p, 0.5, 0.05).run("gmres", **kw)
        assert a["converged"] and b["converged"] and a["outer"] == b["outer"], kw
        assert abs(a["t"] - b["t"]) <= 1e-7 * max(1.0, abs(a["t"]))
        assert np.abs(a["u"] - b["u"]).max() <= 1e-6 * np.abs(a["u"]).max()
        assert len(a["inner_counts"]) == len(b["inner_counts"])
        if kw.get("inner_rule") == "min":
            assert a["inner_total"] >= b["inner_total"]
