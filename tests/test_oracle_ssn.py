"""Pins of the semismooth Newton oracle (Section 5, Algorithm 2) against facts
that do not come from the oracle itself:

* F of the discrete optimality condition equals u minus the textbook proximal
  map of the L^1 penalty with the box (soft threshold, scale by 1/nu, clip);
  the active set is nu times that map's derivative (finite differences);
* the assembled operator with node factors on D_j and E_j equals the C
  oracle's operator;
* the Newton system is the generalized derivative G(u) = I + (1/nu) chi S*S
  (S*S built from per-sample sparse solves, not from the saddle-point matrix);
* beta = 0 without bounds: one Newton step to the linear-quadratic solution;
* beta above every |E[p]|: the control is exactly zero;
* the solution equals the minimizer found by an accelerated proximal gradient
  method on the reduced problem (a different algorithm), with every one of
  the five pieces of F populated;
* Newton steps have the right length (full steps accepted where Newton
  converges locally), and where the line search backtracks it accepts the
  first step of sufficient decrease, with the merit recomputed from
  per-sample solves at the trial control.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import ssn
from oracle.oracle import Oracle
from paper_2302_13680_amd import inputs


def paper_yd(n):
    """y_d = exp(y^2) sin(2 pi x) sin(2 pi y), the target of the paper's experiments."""
    h = 1.0 / (n + 1)
    t = (np.arange(n) + 1.0) * h
    X, Y = np.meshgrid(t, t)
    return np.exp(Y ** 2) * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)


def problem(n=15, N=3, nu=1e-3, seed=3):
    return inputs.make_problem(n, N, nu, M=3, sigma=0.5, decay=True, seed=seed, yd=paper_yd(n), f=0.0)


def prox(w, beta, nu, a, b):
    """argmin over a <= u <= b of nu/2 u^2 - w u + beta |u| (closed form)."""
    return np.clip(np.sign(w) * np.maximum(np.abs(w) - beta, 0.0) / nu, a, b)


@pytest.mark.parametrize("a,b", [(-2.0, 3.0), (-np.inf, np.inf), (-0.5, np.inf)])
def test_F_is_u_minus_proximal_map(a, b):
    rng = np.random.default_rng(0)
    nu, beta = 0.1, 0.3
    w = rng.uniform(-1.5, 1.5, 4000)
    u = rng.standard_normal(4000)
    F = ssn.F_map(u, w, nu, beta, a, b)
    np.testing.assert_allclose(F, u - prox(w, beta, nu, a, b), rtol=0, atol=1e-13)


def test_active_set_is_derivative_of_proximal_map():
    rng = np.random.default_rng(1)
    nu, beta, a, b = 0.1, 0.3, -2.0, 3.0
    w = rng.uniform(-1.5, 1.5, 4000)
    kinks = np.array([-beta, beta, beta + nu * b, nu * a - beta])
    w = w[np.min(np.abs(w[:, None] - kinks[None]), axis=1) > 1e-4]
    eps = 1e-7
    deriv = (prox(w + eps, beta, nu, a, b) - prox(w - eps, beta, nu, a, b)) / (2 * eps)
    np.testing.assert_allclose(ssn.active_set(w, nu, beta, a, b), nu * deriv, atol=1e-6)


def test_assembled_operator_matches_c_oracle_with_node_factors():
    p = problem(n=7, N=3)
    nn = p.n * p.n
    rng = np.random.default_rng(2)
    o = Oracle(p)
    for md, me in [(None, None), (rng.integers(0, 2, nn).astype(float), None),
                   (rng.integers(0, 2, nn).astype(float), rng.uniform(0, 1, nn))]:
        o.set_masks(None if md is None else md.reshape(p.n, p.n), None if me is None else me.reshape(p.n, p.n))
        S = ssn.assemble(p, md, me)
        for _ in range(3):
            v = rng.standard_normal(S.shape[0])
            np.testing.assert_allclose(S @ v, o.apply(v), rtol=1e-13, atol=1e-15)


def reduced_map(p):
    """w(u) = E[p](u) by per-sample sparse solves, and its linear part L_T."""
    n, N = p.n, p.N
    lus = [spla.splu(ssn.stiffness(p, j).tocsc()) for j in range(N)]

    def w_of(u, affine=True):
        w = np.zeros(n * n)
        for j in range(N):
            y = lus[j].solve((p.fP[j].ravel() if affine else 0.0) - p.e[j] * u)
            w += lus[j].solve((p.fY[j].ravel() if affine else 0.0) - p.c[j] * y)
        return w
    return w_of


def test_newton_system_is_generalized_derivative():
    p = problem(n=15, N=3, nu=1e-3)
    n, N, nu = p.n, p.N, p.nu
    nn = n * n
    rng = np.random.default_rng(3)
    u = rng.uniform(-5, 5, nn)
    w_of = reduced_map(p)
    w = w_of(u)
    beta, a, b = 4e-3, -6.0, 6.0
    F = ssn.F_map(u, w, nu, beta, a, b)
    chi = ssn.active_set(w, nu, beta, a, b)
    assert 0.1 < chi.mean() < 0.9
    pn = ssn.newton_problem(p)
    r = np.zeros((2 * N + 1) * nn)
    r[N * nn:(N + 1) * nn] = -pn.g * F
    dx = spla.spsolve(ssn.assemble(pn, md=chi), r)
    du = dx[N * nn:(N + 1) * nn]
    # G(u) du = du - (1/nu) chi L_T du, L_T the linear part of u -> E[p] (= -S*S)
    np.testing.assert_allclose(du - chi * w_of(du, affine=False) / nu, -F, rtol=0, atol=1e-10 * np.abs(F).max())
    # the increments of y and p are the linearized state and adjoint responses
    np.testing.assert_allclose(ssn.expected_p(dx, n, N), w_of(du, affine=False), rtol=0,
                               atol=1e-12 * np.abs(w).max())


def test_initial_state_solves_state_and_adjoint_equations():
    p = problem(n=15, N=3)
    nn = p.n * p.n
    u0 = np.random.default_rng(4).standard_normal(nn)
    x = ssn.initial_state(p, u0)
    r = Oracle(p).residual(x, p.rhs_paper())
    N = p.N
    assert np.abs(r[:N * nn]).max() < 1e-14 and np.abs(r[(N + 1) * nn:]).max() < 1e-14
    np.testing.assert_array_equal(x[N * nn:(N + 1) * nn], u0)


def test_unconstrained_l2_is_one_newton_step_to_lq_solution():
    p = problem(n=15, N=3, nu=1e-4)
    nn = p.n * p.n
    res = ssn.ssn_solve(p, 0.0, -np.inf, np.inf)
    assert res["iterations"] == 1 and res["converged"]
    assert res["chi"].min() == 1.0
    x_lq = spla.spsolve(ssn.assemble(p), p.rhs_paper())
    u_lq = x_lq[p.N * nn:(p.N + 1) * nn]
    np.testing.assert_allclose(res["u"], u_lq, rtol=0, atol=1e-9 * np.abs(u_lq).max())
    np.testing.assert_allclose(res["x"], x_lq, rtol=0, atol=1e-9 * np.abs(x_lq).max())


def test_large_beta_gives_zero_control():
    p = inputs.make_problem(15, 3, 1e-3, M=3, sigma=0.5, decay=True, seed=5, yd=paper_yd(15), f=1.0)
    nn = p.n * p.n
    w0 = ssn.expected_p(ssn.initial_state(p, np.zeros(nn)), p.n, p.N)
    beta = 10 * np.abs(w0).max()
    u0 = 1e-3 * np.random.default_rng(6).standard_normal(nn)
    res = ssn.ssn_solve(p, beta, -1.0, 1.0, u0=u0)
    assert res["iterations"] == 1
    assert np.abs(res["u"]).max() < 1e-15
    for j in range(p.N):
        y = spla.spsolve(ssn.stiffness(p, j).tocsc(), p.fP[j].ravel())
        np.testing.assert_allclose(res["x"][j * nn:(j + 1) * nn], y, rtol=1e-12, atol=1e-15)


def fista(p, beta, a, b, iters=4000, tol=1e-14):
    """Accelerated proximal gradient on the reduced problem
    min 1/2 sum zeta_j |y_j(u) - y_d|_M^2 + nu/2 |u|_M^2 + beta |u|_{L1,M}, a <= u <= b,
    in the M inner product: gradient nu u - E[p](u), prox = clip(soft threshold)."""
    nn = p.n * p.n
    w_of = reduced_map(p)
    v = np.random.default_rng(7).standard_normal(nn)
    for _ in range(60):   # power iteration: Lipschitz constant of the gradient
        v = p.nu * v - w_of(v, affine=False)
        v /= np.linalg.norm(v)
    L = float(v @ (p.nu * v - w_of(v, affine=False)))
    t = 1.0 / (1.02 * L)
    u = np.zeros(nn); z = u.copy(); s = 1.0
    for _ in range(iters):
        g = p.nu * z - w_of(z)
        un = np.clip(np.sign(z - t * g) * np.maximum(np.abs(z - t * g) - t * beta, 0.0), a, b)
        sn = 0.5 * (1 + np.sqrt(1 + 4 * s * s))
        z = un + ((s - 1) / sn) * (un - u)
        if np.abs(un - u).max() < tol:
            return un
        u, s = un, sn
    raise AssertionError("proximal gradient did not converge")


def test_solution_matches_proximal_gradient_on_reduced_problem():
    p = problem(n=15, N=3, nu=1e-3)
    beta, a, b = 4e-3, -6.0, 6.0
    res = ssn.ssn_solve(p, beta, a, b)
    assert res["converged"]
    w = res["w"]
    pieces = [w > beta + p.nu * b, (w >= beta) & (w <= beta + p.nu * b), np.abs(w) < beta,
              (w <= -beta) & (w >= p.nu * a - beta), w < p.nu * a - beta]
    assert all(m.sum() >= 3 for m in pieces), [int(m.sum()) for m in pieces]
    u_ref = fista(p, beta, a, b)
    np.testing.assert_allclose(res["u"], u_ref, rtol=0, atol=1e-9 * np.abs(u_ref).max())


def test_merit_decreases_and_convergence_is_superlinear():
    p = problem(n=15, N=4, nu=1e-4)
    res = ssn.ssn_solve(p, 1e-2, -50.0, 50.0)
    phi = np.array(res["phi"])
    assert res["converged"] and phi[-1] <= 1e-9
    assert np.all(phi[1:] <= (1 - 1e-4) * phi[:-1])
    assert phi[-1] / phi[-2] < 1e-3
    # a Newton step of the right length: every full step is accepted here
    assert res["gammas"] == [1.0] * res["iterations"]


def test_line_search_accepts_the_first_armijo_step():
    """nu = 1e-6: the full Newton step often raises the merit.  Each accepted
    gamma satisfies the sufficient decrease and gamma / rho does not, with the
    merit recomputed from per-sample solves at the trial control (not from the
    increments), and the final state still solves the state and adjoint
    equations of the final control."""
    p = problem(n=15, N=3, nu=1e-6)
    beta, a, b, sigma, rho = 1e-2, -50.0, 50.0, 1e-4, 0.5
    res = ssn.ssn_solve(p, beta, a, b, sigma=sigma, rho=rho, keep_steps=True, maxit=200)
    assert res["converged"]
    assert min(res["gammas"]) < 1.0
    w_of = reduced_map(p)
    h = 1.0 / (p.n + 1)

    def phi(u):
        return ssn.merit(ssn.F_map(u, w_of(u), p.nu, beta, a, b), h)
    for (u, du), g in zip(res["steps"], res["gammas"]):
        ph = phi(u)
        assert phi(u + g * du) - ph <= -sigma * ph + 1e-12 * ph
        if g < 1.0:
            assert phi(u + (g / rho) * du) - ph > -sigma * ph - 1e-12 * ph
    np.testing.assert_allclose(res["w"], w_of(res["u"]), rtol=0, atol=1e-10 * np.abs(res["w"]).max())


@pytest.mark.parametrize("linear", ["vcycle", "gmres"])
def test_multigrid_inner_solves_reach_the_direct_solution(linear):
    p = problem(n=31, N=4, nu=1e-4)
    ref = ssn.ssn_solve(p, 1e-2, -50.0, 50.0)
    res = ssn.ssn_solve(p, 1e-2, -50.0, 50.0, linear=linear)
    assert res["iterations"] == ref["iterations"]
    assert all(k > 1 for k in res["inner"])
    np.testing.assert_allclose(res["u"], ref["u"], rtol=0, atol=1e-9 * np.abs(ref["u"]).max())


def test_invalid_settings_raise():
    p = problem(n=7, N=2)
    with pytest.raises(ValueError):
        ssn.ssn_solve(p, 1e-2, 0.5, 1.0)
    q = inputs.make_problem(7, 2, 1e-3, control_region=(0.25, 0.75, 0.25, 0.75))
    with pytest.raises(ValueError):
        ssn.ssn_solve(q, 1e-2, -1.0, 1.0)


def test_node_factor_coarsening_rules():
    """Injection takes fine node (2X+1, 2K+1); full weighting averages the 3 x 3
    fine nodes with weights (1/4, 1/2, 1/4) per direction: constants are kept
    and x^2 + y^2 becomes x^2 + y^2 + h^2 (h/2 per direction, h the fine spacing),
    level by level."""
    p = problem(n=31, N=2)
    o = Oracle(p)
    n = p.n
    t = (np.arange(n) + 1.0) / (n + 1)
    X, Y = np.meshgrid(t, t)
    q = X ** 2 + Y ** 2
    o.set_masks(np.full((n, n), 0.375), q, coarsen="full")
    hf = 1.0 / (n + 1)
    expect = q
    for l in range(1, o.nlev):
        nl = o.levels_n[l]
        np.testing.assert_array_equal(o.level_factor(l, "d"), np.full((nl, nl), 0.375))
        tc = (np.arange(nl) + 1.0) / (nl + 1)
        Xc, Yc = np.meshgrid(tc, tc)
        h = hf * 2 ** (l - 1)
        expect = expect[1::2, 1::2] + h * h     # the fine level's quadratic plus h^2
        np.testing.assert_allclose(o.level_factor(l, "e"), expect, rtol=0, atol=1e-14)
        if l == 1:   # coarse nodes sit on fine nodes: x_c^2 + y_c^2 + h^2
            np.testing.assert_allclose(expect, Xc ** 2 + Yc ** 2 + hf * hf, rtol=0, atol=1e-15)
    o.set_masks(q, None, coarsen="injection")
    for l in range(1, o.nlev):
        np.testing.assert_array_equal(o.level_factor(l, "d"), o.level_factor(l - 1, "d")[1::2, 1::2])
        assert np.all(o.level_factor(l, "e") == 1.0)


def test_multigrid_inner_counts_are_mesh_independent():
    """With the active set carried to coarse levels by full weighting, the
    V-cycles per Newton step stay bounded as the grid is refined."""
    means = []
    for n in (31, 63):
        p = problem(n=n, N=4, nu=1e-4)
        res = ssn.ssn_solve(p, 1e-2, -50.0, 50.0, linear="vcycle")
        means.append(np.mean(res["inner"]))
    assert max(means) <= 16 and abs(means[1] - means[0]) <= 3, means


def test_solution_matches_proximal_gradient_on_the_lshape():
    """The same independent check on the paper's L-shaped domain (nodes with
    x, y >= 1/2 removed): u stays zero outside, and inside it is the reduced
    problem's minimizer."""
    p = inputs.make_problem(15, 3, 1e-3, M=3, sigma=0.5, decay=True, seed=3, yd=paper_yd(15), f=0.0,
                            domain="lshape")
    beta, a, b = 4e-3, -6.0, 6.0
    res = ssn.ssn_solve(p, beta, a, b)
    assert res["converged"]
    outside = p.domain.ravel() == 0
    assert np.all(res["u"][outside] == 0)
    u_ref = fista(p, beta, a, b)
    np.testing.assert_allclose(res["u"], u_ref, rtol=0, atol=1e-9 * np.abs(u_ref).max())
