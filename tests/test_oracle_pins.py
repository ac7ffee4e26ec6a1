"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself: a
closed form, a textbook spectrum, a dense library solve, a structural
property of S, or the convergence theory of Section 3.1.
"""
import math

import numpy as np
import pytest

from paper_2302_13680_amd import inputs


def _rand_problem(n, N, seed=0, nu=1e-4, sigma=0.5, M=4):
    return inputs.make_problem(n, N, nu, M=M, sigma=sigma, decay=False, seed=seed)


def _sine_mode(n, m, l):
    h = 1.0 / (n + 1)
    xs = (np.arange(n) + 1) * h
    X, Y = np.meshgrid(xs, xs)
    return np.sin(m * math.pi * X) * np.sin(l * math.pi * Y)


# --------------------------------------------------------------------- operator
def test_apply_constant_kappa_matches_textbook_laplacian(oracle_mod):
    """kappa = 1: A is the h^2-scaled 5-point Laplacian with eigenvalues
    4 sin^2(m pi h/2) + 4 sin^2(l pi h/2) on the sine modes; the blocks of S
    must act on single-field inputs as eq. (2) places them."""
    n, N = 15, 3
    p = inputs.make_problem(n, N, 1e-3, kappa_const=1.0)
    o = oracle_mod.Oracle(p)
    h = 1.0 / (n + 1)
    nn = n * n
    for (m, l) in [(1, 1), (2, 5), (7, 3)]:
        phi = _sine_mode(n, m, l).ravel()
        lam = 4 * math.sin(m * math.pi * h / 2) ** 2 + 4 * math.sin(l * math.pi * h / 2) ** 2
        for j in range(N):
            # y_j only: Y row gets C_j y, P row gets A_j y
            x = np.zeros(o.vlen()); x[j * nn:(j + 1) * nn] = phi
            out = o.apply(x)
            np.testing.assert_allclose(out[j * nn:(j + 1) * nn], p.c[j] * phi, atol=1e-14)
            np.testing.assert_allclose(out[(N + 1 + j) * nn:(N + 2 + j) * nn], lam * phi, atol=1e-12)
            assert np.abs(out[N * nn:(N + 1) * nn]).max() == 0.0
            # p_j only: Y row gets A_j^T p, U row gets D_j p
            x = np.zeros(o.vlen()); x[(N + 1 + j) * nn:(N + 2 + j) * nn] = phi
            out = o.apply(x)
            np.testing.assert_allclose(out[j * nn:(j + 1) * nn], lam * phi, atol=1e-12)
            np.testing.assert_allclose(out[N * nn:(N + 1) * nn], p.d[j] * phi, atol=1e-14)
        # u only: U row gets G u, every P row gets E_j u
        x = np.zeros(o.vlen()); x[N * nn:(N + 1) * nn] = phi
        out = o.apply(x)
        np.testing.assert_allclose(out[N * nn:(N + 1) * nn], p.g * phi, atol=1e-14)
        for j in range(N):
            np.testing.assert_allclose(out[(N + 1 + j) * nn:(N + 2 + j) * nn], p.e[j] * phi, atol=1e-14)


def test_assembled_S_is_symmetric(oracle_mod):
    """The rescaled system is symmetric (end of Section 2); a transposed face
    index or a misplaced block breaks it."""
    for (n, N) in [(7, 1), (7, 3)]:
        o = oracle_mod.Oracle(_rand_problem(n, N, seed=3), coarsest_n=3)
        S = o.assemble()
        assert np.abs(S - S.T).max() <= 1e-15 * np.abs(S).max()


def test_stiffness_energy_identity(oracle_mod):
    """Summation by parts: y^T A_j y = sum over faces of kappa_f (y_left - y_right)^2,
    with zero values outside the grid."""
    n, N = 7, 2
    p = _rand_problem(n, N, seed=5)
    o = oracle_mod.Oracle(p, coarsest_n=3)
    nn = n * n
    rng = np.random.default_rng(0)
    for j in range(N):
        y = rng.standard_normal((n, n))
        x = np.zeros(o.vlen()); x[j * nn:(j + 1) * nn] = y.ravel()
        Ay = o.apply(x)[(N + 1 + j) * nn:(N + 2 + j) * nn]
        ypad = np.zeros((n + 2, n + 2)); ypad[1:-1, 1:-1] = y
        energy = 0.0
        for k in range(n):
            for f in range(n + 1):
                energy += p.kx[j, k, f] * (ypad[k + 1, f + 1] - ypad[k + 1, f]) ** 2
        for gg in range(n + 1):
            for xx in range(n):
                energy += p.ky[j, gg, xx] * (ypad[gg + 1, xx + 1] - ypad[gg, xx + 1]) ** 2
        assert abs(float(y.ravel() @ Ay) - energy) <= 1e-12 * energy


def test_stiffness_row_sums_are_boundary_faces(oracle_mod):
    """A_j 1 vanishes in the interior and equals the boundary faces next to the
    boundary (conservation of the flux form)."""
    n, N = 7, 2
    p = _rand_problem(n, N, seed=6)
    o = oracle_mod.Oracle(p, coarsest_n=3)
    nn = n * n
    for j in range(N):
        x = np.zeros(o.vlen()); x[j * nn:(j + 1) * nn] = 1.0
        rs = o.apply(x)[(N + 1 + j) * nn:(N + 2 + j) * nn].reshape(n, n)
        expect = np.zeros((n, n))
        expect[:, 0] += p.kx[j, :, 0]
        expect[:, -1] += p.kx[j, :, n]
        expect[0, :] += p.ky[j, 0, :]
        expect[-1, :] += p.ky[j, n, :]
        np.testing.assert_allclose(rs, expect, atol=1e-13)


# ------------------------------------------------------------------- node solve
def test_node_solve_matches_dense_lu_of_reduced_block(oracle_mod):
    """eq. solution_reduced_system against a dense solve of eq. reduced_matrices."""
    rng = np.random.default_rng(1)
    for N in [1, 2, 7, 33]:
        a = rng.uniform(0.5, 3.0, N); c = rng.uniform(0.1, 2.0, N)
        d = rng.uniform(-2.0, -0.1, N); e = rng.uniform(-2.0, -0.1, N); g = rng.uniform(0.1, 1.0)
        S = np.zeros((2 * N + 1, 2 * N + 1))
        S[:N, :N] = np.diag(c); S[:N, N + 1:] = np.diag(a)
        S[N, N] = g; S[N, N + 1:] = d
        S[N + 1:, :N] = np.diag(a); S[N + 1:, N] = e
        b = rng.standard_normal(2 * N + 1)
        ref = np.linalg.solve(S, b)
        y, u, p = oracle_mod.node_solve(a, c, d, e, g, b[:N], b[N], b[N + 1:])
        got = np.concatenate([y, [u], p])
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_node_blocks_probed_from_S_have_paper_structure(oracle_mod):
    """R_i S P_i probed from the operator has the structure of eq. reduced_matrices
    with a_j = (A_j)_ii, and the denominator of eq. solution_reduced_system is
    G_ii + (M)^3_ii sum_j zeta_j (A_j)_ii^{-2} > 0."""
    n, N = 7, 3
    p = _rand_problem(n, N, seed=7)
    o = oracle_mod.Oracle(p, coarsest_n=3)
    S = o.assemble()
    nn = n * n
    h = p.h
    for i in [0, 10, 24, 48]:
        idx = [j * nn + i for j in range(N)] + [N * nn + i] + [(N + 1 + j) * nn + i for j in range(N)]
        Si = S[np.ix_(idx, idx)]
        a = np.diag(Si[N + 1:, :N])
        np.testing.assert_allclose(Si[:N, N + 1:], np.diag(a), atol=0)
        np.testing.assert_allclose(Si[:N, :N], np.diag(p.c), atol=0)
        assert Si[N, N] == p.g
        np.testing.assert_allclose(Si[N, N + 1:], p.d, atol=0)
        np.testing.assert_allclose(Si[N + 1:, N], p.e, atol=0)
        k, x = divmod(i, n)
        for j in range(N):
            diag = p.kx[j, k, x] + p.kx[j, k, x + 1] + p.ky[j, k, x] + p.ky[j, k + 1, x]
            assert abs(a[j] - diag) <= 1e-15 * diag
        den = p.g + np.sum(p.d * p.c * p.e / a ** 2)
        den_paper = p.g + (h * h) ** 3 * np.sum((1.0 / N) * a ** -2.0)
        assert den > 0 and abs(den - den_paper) <= 1e-13 * den


def test_red_halfsweep_zeroes_red_residual(oracle_mod):
    """Gauss-Seidel with theta = 1 solves every red node exactly given its black
    neighbours: after a red half-sweep all 2N+1 residual rows of every red node
    vanish and the black nodes are untouched."""
    n, N = 15, 4
    p = _rand_problem(n, N, seed=8)
    o = oracle_mod.Oracle(p)
    rng = np.random.default_rng(2)
    x0 = rng.standard_normal(o.vlen())
    f = p.rhs_paper()
    for colour in (0, 1):
        x1 = o.halfsweep(x0, f, colour)
        r = o.residual(x1, f).reshape(2 * N + 1, n, n)
        kk, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        act = ((kk + xx) % 2) == colour
        scale = np.abs(o.residual(x0, f)).max()
        assert np.abs(r[:, act]).max() <= 1e-12 * scale
        unchanged = (x1 - x0).reshape(2 * N + 1, n, n)[:, ~act]
        assert np.abs(unchanged).max() == 0.0


def test_sample_permutation_equivariance(oracle_mod):
    """Permuting the samples permutes y_j and p_j and leaves u unchanged."""
    n, N = 15, 5
    p = _rand_problem(n, N, seed=9)
    perm = np.array([3, 0, 4, 1, 2])
    q = inputs.make_problem(n, N, p.nu, M=4, sigma=0.5, xi=p.xi[perm])
    o1, o2 = oracle_mod.Oracle(p), oracle_mod.Oracle(q)
    x1 = o1.vcycle(np.zeros(o1.vlen()), p.rhs_paper(), 2).reshape(2 * N + 1, -1)
    x2 = o2.vcycle(np.zeros(o2.vlen()), q.rhs_paper(), 2).reshape(2 * N + 1, -1)
    np.testing.assert_allclose(x2[:N], x1[:N][perm], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(x2[N + 1:], x1[N + 1:][perm], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(x2[N], x1[N], rtol=1e-11, atol=1e-14)


# -------------------------------------------------------------------- transfers
def test_prolongation_mode_action_matches_paper(oracle_mod):
    """eq. action_restriction_prolongation, per dimension: linear interpolation maps
    the coarse mode phi_j to c_j^2 phi_j - s_j^2 phi_{Nh+1-j}; the 2D bilinear P is
    the tensor product."""
    nf = 15
    nc = 7
    h = 1.0 / (nf + 1)
    N = 1
    for (j, l) in [(1, 1), (2, 3), (7, 5)]:
        coarse = np.zeros((2 * N + 1) * nc * nc)
        phic = _sine_mode(nc, j, l)          # sin(2 I j pi h) on the coarse grid
        coarse[nc * nc:2 * nc * nc] = phic.ravel()   # the U field
        fine = oracle_mod.prolong_add(nc, N, coarse, np.zeros((2 * N + 1) * nf * nf))
        cj2, sj2 = math.cos(j * math.pi * h / 2) ** 2, math.sin(j * math.pi * h / 2) ** 2
        cl2, sl2 = math.cos(l * math.pi * h / 2) ** 2, math.sin(l * math.pi * h / 2) ** 2
        jt, lt = nf + 1 - j, nf + 1 - l
        expect = (cj2 * cl2 * _sine_mode(nf, j, l) - sj2 * cl2 * _sine_mode(nf, jt, l)
                  - cj2 * sl2 * _sine_mode(nf, j, lt) + sj2 * sl2 * _sine_mode(nf, jt, lt))
        got = fine[nf * nf:2 * nf * nf].reshape(nf, nf)
        np.testing.assert_allclose(got, expect, atol=1e-13)
        assert np.abs(fine[:nf * nf]).max() == 0 and np.abs(fine[2 * nf * nf:]).max() == 0


def test_restriction_is_transpose_and_mode_action(oracle_mod):
    """R = P^T (checked through inner products) and, per dimension,
    R(e_j phi_j + e_jt phi_jt) = 2 (c_j^2 e_j - s_j^2 e_jt) phi^c_j: the printed
    stencil [1/2 1 1/2] acting on the modes (twice the scaling of the paper's
    mode formula; the two-level operator is invariant to it)."""
    nf, nc, N = 15, 7, 2
    rng = np.random.default_rng(4)
    a = rng.standard_normal((2 * N + 1) * nf * nf)
    b = rng.standard_normal((2 * N + 1) * nc * nc)
    Ra = oracle_mod.restrict(nf, N, a)
    Pb = oracle_mod.prolong_add(nc, N, b, np.zeros_like(a))
    assert abs(Ra @ b - a @ Pb) <= 1e-12 * np.abs(a).sum()
    h = 1.0 / (nf + 1)
    j, l = 3, 2
    ej, ejt = 0.7, -1.3
    jt = nf + 1 - j
    fine = np.zeros((2 * N + 1) * nf * nf)
    fine[:nf * nf] = (ej * _sine_mode(nf, j, l) + ejt * _sine_mode(nf, jt, l)).ravel()
    got = oracle_mod.restrict(nf, N, fine)[:nc * nc].reshape(nc, nc)
    cj2, sj2 = math.cos(j * math.pi * h / 2) ** 2, math.sin(j * math.pi * h / 2) ** 2
    cl2 = math.cos(l * math.pi * h / 2) ** 2
    expect = 2 * (cj2 * ej - sj2 * ejt) * 2 * cl2 * _sine_mode(nc, j, l)
    np.testing.assert_allclose(got, expect, atol=1e-13)


def test_face_coarsening_reproduces_linear_fields(oracle_mod):
    """Averaging the two fine faces under a coarse face is exact for a coefficient
    linear in position: the coarse faces equal the field at the coarse face
    midpoints (rediscretization on the coarse mesh)."""
    nf, N = 15, 2
    nc = 7
    hf, hc = 1.0 / (nf + 1), 1.0 / (nc + 1)
    kap = lambda x, y, j: 1.0 + 0.3 * x + 0.7 * y + 0.1 * j
    kx = np.array([[[kap((f + 0.5) * hf, (k + 1) * hf, j) for f in range(nf + 1)] for k in range(nf)] for j in range(N)])
    ky = np.array([[[kap((x + 1) * hf, (g + 0.5) * hf, j) for x in range(nf)] for g in range(nf + 1)] for j in range(N)])
    kxc, kyc = oracle_mod.coarsen_faces(nf, N, kx, ky)
    ex = np.array([[[kap((F + 0.5) * hc, (K + 1) * hc, j) for F in range(nc + 1)] for K in range(nc)] for j in range(N)])
    ey = np.array([[[kap((X + 1) * hc, (G + 0.5) * hc, j) for X in range(nc)] for G in range(nc + 1)] for j in range(N)])
    np.testing.assert_allclose(kxc, ex, atol=1e-14)
    np.testing.assert_allclose(kyc, ey, atol=1e-14)


# ------------------------------------------------------------------ coarse solve
@pytest.mark.parametrize("N", [1, 3, 6])
def test_coarse_solve_matches_dense_solve(oracle_mod, N):
    p = _rand_problem(7, N, seed=10 + N)
    o = oracle_mod.Oracle(p, coarsest_n=7)
    assert o.nlev == 1
    S = o.assemble()
    F = np.random.default_rng(N).standard_normal(o.vlen())
    ref = np.linalg.solve(S, F)
    got = o.coarse_solve(F)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


# -------------------------------------------------------------- whole solutions
@pytest.mark.parametrize("n,N,nu", [(7, 3, 1e-4), (31, 8, 1e-4), (15, 1, 1e-2)])
def test_closed_form_solution_constant_kappa(oracle_mod, n, N, nu):
    """kappa = 1, f = 0, y_d = sin(pi x) sin(pi y), the (1,1) eigenmode of A with
    eigenvalue lam = 8 sin^2(pi h/2).  Then y_j = alpha phi, p_j = beta phi,
    u = gamma phi with beta = h^2 lam / (N (lam^2 + h^4/nu)), gamma = N beta/nu,
    alpha = h^2 gamma / lam (from the three block rows of eq. (2))."""
    p = inputs.make_problem(n, N, nu, kappa_const=1.0, f=0.0)
    o = oracle_mod.Oracle(p, coarsest_n=3 if n > 3 else 1)
    h = p.h
    lam = 8 * math.sin(math.pi * h / 2) ** 2
    beta = h * h * lam / (N * (lam ** 2 + h ** 4 / nu))
    gamma = N * beta / nu
    alpha = h * h * gamma / lam
    phi = _sine_mode(n, 1, 1).ravel()
    # with f = 0 the right-hand side is small (h^2/N) against S, so the rounding
    # floor of the relative residual sits near 1e-12
    x, its, _ = o.solve_vcycle(p.rhs_paper(), tol=1e-11, maxit=100)
    assert its > 0
    X = x.reshape(2 * N + 1, n * n)
    for j in range(N):
        np.testing.assert_allclose(X[j], alpha * phi, rtol=1e-8, atol=1e-10 * alpha)
        np.testing.assert_allclose(X[N + 1 + j], beta * phi, rtol=1e-8, atol=1e-10 * beta)
    np.testing.assert_allclose(X[N], gamma * phi, rtol=1e-8, atol=1e-10 * gamma)


@pytest.mark.parametrize("n,N", [(7, 2), (15, 2), (15, 3)])
def test_vcycle_and_gmres_converge_to_dense_solution(oracle_mod, n, N):
    p = _rand_problem(n, N, seed=20 + n + N)
    o = oracle_mod.Oracle(p, coarsest_n=3)
    S = o.assemble()
    f = p.rhs_paper()
    xs = np.linalg.solve(S, f)
    xv, its, _ = o.solve_vcycle(f, tol=1e-13, maxit=100)
    xg, itg, _ = o.gmres(f, m=30, tol=1e-13, maxit=100)
    assert its > 0 and itg > 0
    assert itg <= its
    for x in (xv, xg):
        assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)


def test_sample_invariance_of_identical_samples(oracle_mod):
    """With identical coefficients in every sample, y_j are identical, (u, y) do
    not depend on N and N p_j does not either (zeta = 1/N); N = 1 is the
    deterministic collective method (remark on the deterministic setting)."""
    n = 15
    xi1 = np.array([[0.3, -1.1, 0.4, 0.8]])
    sols = {}
    for N in (1, 4):
        p = inputs.make_problem(n, N, 1e-4, M=4, sigma=0.5, xi=np.repeat(xi1, N, axis=0))
        o = oracle_mod.Oracle(p)
        x, its, _ = o.solve_vcycle(p.rhs_paper(), tol=1e-13, maxit=100)
        sols[N] = x.reshape(2 * N + 1, n * n)
    y1, u1, p1 = sols[1][0], sols[1][1], sols[1][2]
    X4 = sols[4]
    for j in range(4):
        np.testing.assert_allclose(X4[j], y1, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(4 * X4[5 + j], p1, rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(X4[4], u1, rtol=1e-9, atol=1e-12)


def test_mesh_independent_contraction(oracle_mod):
    """Iteration counts of the stationary V-cycle stay constant as the mesh is
    refined (Table 1, row N_h): geometric-mean contraction bounded and counts
    within +-2."""
    counts, rates = [], []
    for n in (15, 31, 63, 127):
        p = inputs.make_problem(n, 4, 1e-4, M=6, sigma=0.5, decay=True, seed=11)
        o = oracle_mod.Oracle(p)
        _, its, hist = o.solve_vcycle(p.rhs_paper(), tol=1e-10, maxit=60)
        assert its > 0
        counts.append(its)
        rates.append((hist[-1] / hist[1]) ** (1.0 / (len(hist) - 2)))
    assert max(counts) - min(counts) <= 2, counts
    assert max(rates) < 0.2, rates


def test_robust_in_nu_and_N(oracle_mod):
    """Counts stay bounded over nu in [1e-8, 1e-2] and over N (Table 1 rows nu, N)."""
    counts = []
    for nu in (1e-2, 1e-4, 1e-6, 1e-8):
        p = inputs.make_problem(31, 8, nu, M=6, sigma=0.5, decay=True, seed=12)
        _, its, _ = oracle_mod.Oracle(p).solve_vcycle(p.rhs_paper(), tol=1e-10, maxit=60)
        counts.append(its)
    for N in (2, 16, 64):
        p = inputs.make_problem(31, N, 1e-4, M=6, sigma=0.5, decay=True, seed=13)
        _, its, _ = oracle_mod.Oracle(p).solve_vcycle(p.rhs_paper(), tol=1e-10, maxit=60)
        counts.append(its)
    assert all(0 < c <= 20 for c in counts), counts


def test_fp32_refinement_reaches_fp64_tolerance(oracle_mod):
    """The FP32 V-cycle inside FP64 refinement reaches 1e-10 and agrees with the
    FP64 solution to the accuracy the residual bound allows."""
    p = inputs.small_fp64()
    o = oracle_mod.Oracle(p)
    f = p.rhs_paper()
    x64, _, _ = o.gmres(f, tol=1e-12)
    for m in (30, 0):
        x, its, inner, hist = o.solve_ir(f, tol=1e-10, m=m)
        assert its > 0 and hist[-1] <= 1e-10
        assert np.linalg.norm(x - x64) <= 1e-6 * np.linalg.norm(x64)
    # a single FP32 cycle agrees with the FP64 cycle to FP32 accuracy
    x1 = o.vcycle(np.zeros(o.vlen()), f, 1)
    x2 = o.vcycle32(np.zeros(o.vlen()), f, 1)
    assert np.linalg.norm(x1 - x2) <= 1e-5 * np.linalg.norm(x1)
