"""Stochastic collocation (the paper's SC columns: tensor Gauss-Hermite nodes in
M = 3 normal variables, N = q^M, weights zeta_j): pins of the quadrature rule
against the moments of the normal distribution, of how the weights enter the
system, and of the solver's robustness in N (Table 1, SC rows)."""
import math

import numpy as np
import pytest

from paper_2302_13680_amd import inputs


@pytest.mark.parametrize("q", [2, 3, 4, 5])
def test_gauss_hermite_rule_reproduces_normal_moments(q):
    """A q-point rule per variable integrates polynomials of degree <= 2q - 1 in
    each variable exactly: E[xi^k] = (k-1)!! for even k, 0 for odd k, and the
    variables are independent."""
    M = 3
    xi, zeta = inputs.stochastic_collocation(M, q)
    assert xi.shape == (q ** M, M) and zeta.shape == (q ** M,)
    assert np.all(zeta > 0) and abs(zeta.sum() - 1.0) <= 1e-14
    for k in range(0, 2 * q):
        exact = 0.0 if k % 2 else float(math.prod(range(k - 1, 0, -2)))
        for m in range(M):
            assert abs(np.sum(zeta * xi[:, m] ** k) - exact) <= 1e-12 * max(1.0, exact), (q, k, m)
    assert abs(np.sum(zeta * xi[:, 0] * xi[:, 1])) <= 1e-14
    assert abs(np.sum(zeta * xi[:, 0] ** 2 * xi[:, 2] ** 2) - 1.0) <= 1e-13


def test_collocation_weights_enter_as_quadrature_weights(oracle_mod):
    """With the same coefficient in every sample, the weighted system has y_j and
    the unscaled adjoints p_j = p^_j / zeta_j identical across j and equal to
    the N = 1 solution, and u does not depend on the rule (the weights sum to 1)."""
    n = 15
    sols = {}
    for q in (1, 3):
        xi, zeta = inputs.stochastic_collocation(2, q)
        p = inputs.make_problem(n, xi.shape[0], 1e-4, M=2, kappa_const=1.0, xi=xi, weights=zeta)
        x, its, _ = oracle_mod.Oracle(p).solve_vcycle(p.rhs_paper(), tol=1e-13, maxit=100)
        assert its > 0
        sols[q] = (x.reshape(2 * p.N + 1, n * n), zeta)
    X1, _ = sols[1]
    X9, zeta = sols[3]
    N = len(zeta)
    for j in range(N):
        np.testing.assert_allclose(X9[j], X1[0], rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(X9[N + 1 + j] / zeta[j], X1[2], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(X9[N], X1[1], rtol=1e-9, atol=1e-12)


def test_collocation_system_is_symmetric_and_solved(oracle_mod):
    p = inputs.collocation_problem(7, 2, M=3)          # N = 8
    o = oracle_mod.Oracle(p, coarsest_n=3)
    S = o.assemble()
    assert np.abs(S - S.T).max() <= 1e-15 * np.abs(S).max()
    f = p.rhs_paper()
    xs = np.linalg.solve(S, f)
    xv, its, _ = o.solve_vcycle(f, tol=1e-13, maxit=100)
    xg, itg, _ = o.gmres(f, m=30, tol=1e-13, maxit=100)
    assert its > 0 and 0 < itg <= its
    for x in (xv, xg):
        assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)


def test_collocation_counts_robust_in_N(oracle_mod):
    """V(2,2) counts over N = 8, 27, 64, 125 collocation points stay within +-2."""
    counts = []
    for q in (2, 3, 4, 5):
        p = inputs.collocation_problem(31, q, M=3)
        _, its, _ = oracle_mod.Oracle(p).solve_vcycle(p.rhs_paper(), tol=1e-9, maxit=60)
        assert its > 0
        counts.append(its)
    assert max(counts) - min(counts) <= 2, counts
