"""Local control (the paper's Section 3.2 square-domain experiment with the control
acting on (0.25, 0.75)^2; eq. solution_reduced_system2 at nodes without
control): pins of the oracle's control mask against dense algebra built here."""
import numpy as np
import pytest

from paper_2302_13680_amd import inputs

REGION = (0.25, 0.75, 0.25, 0.75)


def _prob(n, N, seed, region=REGION, **kw):
    return inputs.make_problem(n, N, 1e-4, M=4, sigma=0.5, decay=False, seed=seed, control_region=region, **kw)


def _stiffness(p, j):
    """Textbook 5-point matrix of sample j from the face arrays (independent of
    the oracle's stencil code)."""
    n = p.n
    A = np.zeros((n * n, n * n))
    for k in range(n):
        for x in range(n):
            i = k * n + x
            kw, ke, ks, kn = p.kx[j, k, x], p.kx[j, k, x + 1], p.ky[j, k, x], p.ky[j, k + 1, x]
            A[i, i] = kw + ke + ks + kn
            if x > 0: A[i, i - 1] = -kw
            if x < n - 1: A[i, i + 1] = -ke
            if k > 0: A[i, i - n] = -ks
            if k < n - 1: A[i, i + n] = -kn
    return A


def test_mask_region_is_the_closed_square():
    p = _prob(31, 2, seed=1)
    h = 1.0 / 32
    nodes = (np.arange(31) + 1) * h
    inside = (nodes >= 0.25 - 1e-12) & (nodes <= 0.75 + 1e-12)
    np.testing.assert_array_equal(p.ctrl, np.outer(inside, inside).astype(float))
    assert p.ctrl.sum() == 17 * 17


def test_masked_operator_scales_the_control_couplings(oracle_mod):
    """S with a mask equals S without one except that the couplings between u_i
    and p_j,i carry the factor m_i, in both directions (S stays symmetric)."""
    n, N = 7, 2
    p = _prob(n, N, seed=3, region=(0.3, 0.7, 0.2, 0.6))
    q = _prob(n, N, seed=3, region=None)
    Sm = oracle_mod.Oracle(p, coarsest_n=3).assemble()
    Sf = oracle_mod.Oracle(q, coarsest_n=3).assemble()
    nn = n * n
    mask = p.ctrl.ravel()
    expect = Sf.copy()
    for i in range(nn):
        for j in range(N):
            expect[N * nn + i, (N + 1 + j) * nn + i] *= mask[i]
            expect[(N + 1 + j) * nn + i, N * nn + i] *= mask[i]
    np.testing.assert_array_equal(Sm, expect)
    assert np.array_equal(Sm, Sm.T)


def test_full_mask_is_the_unmasked_method(oracle_mod):
    p = _prob(31, 3, seed=5, region=(0.0, 1.0, 0.0, 1.0))
    q = _prob(31, 3, seed=5, region=None)
    assert p.ctrl.min() == 1.0
    f = p.rhs_paper()
    xa = oracle_mod.Oracle(p).vcycle(np.zeros(f.size), f, 2)
    xb = oracle_mod.Oracle(q).vcycle(np.zeros(f.size), f, 2)
    np.testing.assert_array_equal(xa, xb)


def test_no_control_decouples_the_samples(oracle_mod):
    """With the mask zero everywhere u = 0 and every sample solves its own two
    PDEs: A_j y_j = f_P,j, A_j p_j = f_Y,j - C_j y_j."""
    n, N = 15, 3
    p = _prob(n, N, seed=6, region=(2.0, 3.0, 2.0, 3.0))
    assert p.ctrl.max() == 0.0
    x, its, _ = oracle_mod.Oracle(p).solve_vcycle(p.rhs_paper(), tol=1e-13, maxit=100)
    assert its > 0
    X = x.reshape(2 * N + 1, n * n)
    assert np.abs(X[N]).max() == 0.0
    for j in range(N):
        A = _stiffness(p, j)
        y = np.linalg.solve(A, p.fP[j].ravel())
        pj = np.linalg.solve(A, p.fY[j].ravel() - p.c[j] * y)
        assert np.linalg.norm(X[j] - y) <= 1e-11 * np.linalg.norm(y)
        assert np.linalg.norm(X[N + 1 + j] - pj) <= 1e-11 * np.linalg.norm(pj)


@pytest.mark.parametrize("smoother,theta", [("gs", 1.0), ("jacobi", 0.5)])
def test_local_control_converges_to_dense_solution(oracle_mod, smoother, theta):
    n, N = 15, 2
    p = _prob(n, N, seed=7)
    o = oracle_mod.Oracle(p, coarsest_n=3, smoother=smoother, theta=theta)
    S = o.assemble()
    f = p.rhs_paper()
    xs = np.linalg.solve(S, f)
    xv, its, _ = o.solve_vcycle(f, tol=1e-13, maxit=200)
    xg, itg, _ = o.gmres(f, m=30, tol=1e-13, maxit=200)
    assert its > 0 and 0 < itg <= its
    for x in (xv, xg):
        assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)
    # the control vanishes where it does not act (f_U = 0 there)
    U = xs.reshape(2 * N + 1, n * n)[N]
    assert np.abs(U[p.ctrl.ravel() == 0]).max() <= 1e-13 * np.abs(U).max()


def test_gauss_seidel_cycles_keep_the_control_off_support(oracle_mod):
    """theta = 1: every half-sweep solves a node without control exactly, so u is
    exactly zero there after each V-cycle (eq. solution_reduced_system2)."""
    p = _prob(31, 4, seed=8)
    o = oracle_mod.Oracle(p)
    f = p.rhs_paper()
    x = np.zeros(f.size)
    off = p.ctrl.ravel() == 0
    for _ in range(3):
        x = o.vcycle(x, f, 1)
        U = x.reshape(2 * p.N + 1, -1)[p.N]
        assert np.abs(U[off]).max() == 0.0 and np.abs(U[~off]).max() > 0.0


def test_local_control_counts_mesh_independent(oracle_mod):
    counts = []
    for n in (31, 63, 127):
        p = inputs.make_problem(n, 4, 1e-4, M=6, sigma=0.5, decay=True, seed=9, control_region=REGION)
        _, its, _ = oracle_mod.Oracle(p).solve_vcycle(p.rhs_paper(), tol=1e-9, maxit=100)
        assert its > 0
        counts.append(its)
    assert max(counts) - min(counts) <= 2, counts


@pytest.mark.parametrize("N", [1, 3])
def test_masked_coarse_solve_is_a_dense_solve(oracle_mod, N):
    """The coarsest direct solve with a mask (block elimination through the
    masked control Schur complement) against a dense solve of that level."""
    p = _prob(15, N, seed=10 + N)
    o = oracle_mod.Oracle(p, coarsest_n=7)
    l = o.nlev - 1
    S = o.assemble(l)
    F = np.random.default_rng(N).standard_normal(o.vlen(l))
    ref = np.linalg.solve(S, F)
    assert np.linalg.norm(o.coarse_solve(F) - ref) <= 1e-11 * np.linalg.norm(ref)


def test_control_space_transfer(oracle_mod):
    """The U block moves between levels within the control space (the control
    lives on the region's nodes only): the oracle's coarse right-hand side and
    correction equal the plain full-weighting restriction and bilinear
    prolongation with the U entries of nodes outside the region dropped (the
    coarse node keeping the region of the fine node it coincides with), and the
    two are transposes of each other on the U block."""
    n, N = 31, 3
    p = _prob(n, N, seed=7)
    o = oracle_mod.Oracle(p)
    rng = np.random.default_rng(3)
    nc, nn, nnc = 15, n * n, 15 * 15
    ctrl = p.ctrl.reshape(nn) != 0
    cctrl = p.ctrl[1::2, 1::2].reshape(nnc) != 0
    x = rng.standard_normal(o.vlen(0))
    f = rng.standard_normal(o.vlen(0))
    r = o.residual(x, f)
    r[N * nn:(N + 1) * nn] *= ctrl
    want = oracle_mod.restrict(n, N, r)
    want[N * nnc:(N + 1) * nnc] *= cctrl
    np.testing.assert_allclose(o.residual_restrict(x, f), want, rtol=0, atol=1e-13 * np.abs(want).max())
    c = rng.standard_normal(o.vlen(1))
    fine = rng.standard_normal(o.vlen(0))
    plain = oracle_mod.prolong_add(nc, N, c, fine)
    got = o.prolong_control(c, fine)
    keep = np.concatenate([np.ones(N * nn, bool), ctrl, np.ones(N * nn, bool)])
    np.testing.assert_array_equal(got[keep], plain[keep])
    np.testing.assert_array_equal(got[~keep], fine[~keep])
    # <R r, c>_U = <r, P c>_U for c zero at coarse nodes without a control
    cU = c[N * nnc:(N + 1) * nnc] * cctrl
    cz = np.zeros_like(c)
    cz[N * nnc:(N + 1) * nnc] = cU
    Rr = o.residual_restrict(np.zeros(o.vlen(0)), f)[N * nnc:(N + 1) * nnc]
    Pc = o.prolong_control(cz, np.zeros(o.vlen(0)))[N * nn:(N + 1) * nn]
    assert abs(Rr @ cU - f[N * nn:(N + 1) * nn] @ Pc) <= 1e-12 * np.abs(Rr).sum() * np.abs(cU).max()
