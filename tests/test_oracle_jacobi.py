"""Pins of the oracle's damped collective Jacobi smoother (eq. collective_smoothing
as printed: x <- x + theta sum_i P_i S~_i^{-1} R_i (f - S x)), the smoother of
the paper's experiments with theta = 1/2 (Section 3.2).  Each check compares
with a dense computation or with the convergence behaviour the paper reports."""
import numpy as np
import pytest

from paper_2302_13680_amd import inputs


def _rand_problem(n, N, seed=0, nu=1e-4):
    return inputs.make_problem(n, N, nu, M=4, sigma=0.5, decay=False, seed=seed)


def _node_indices(n, N, i):
    nn = n * n
    return [j * nn + i for j in range(N)] + [N * nn + i] + [(N + 1 + j) * nn + i for j in range(N)]


@pytest.mark.parametrize("n,N,theta", [(3, 2, 0.5), (7, 3, 0.5), (7, 1, 1.0)])
def test_jacobi_step_is_the_block_diagonal_definition(oracle_mod, n, N, theta):
    """The step equals x + theta D^{-1} (f - S x) with D the block diagonal of the
    assembled S over the nodes (each block a dense (2N+1)x(2N+1) solve)."""
    p = _rand_problem(n, N, seed=n + N)
    o = oracle_mod.Oracle(p, coarsest_n=1 if n == 3 else 3)
    S = o.assemble()
    rng = np.random.default_rng(n * N)
    x = rng.standard_normal(o.vlen())
    f = rng.standard_normal(o.vlen())
    r = f - S @ x
    ref = x.copy()
    for i in range(n * n):
        idx = _node_indices(n, N, i)
        ref[idx] += theta * np.linalg.solve(S[np.ix_(idx, idx)], r[idx])
    got = o.jacobi(x, f, theta)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,N", [(7, 2), (15, 3)])
def test_jacobi_vcycle_and_gmres_converge_to_dense_solution(oracle_mod, n, N):
    p = _rand_problem(n, N, seed=30 + n + N)
    o = oracle_mod.Oracle(p, coarsest_n=3, theta=0.5, smoother="jacobi")
    S = o.assemble()
    f = p.rhs_paper()
    xs = np.linalg.solve(S, f)
    xv, its, _ = o.solve_vcycle(f, tol=1e-13, maxit=200)
    xg, itg, _ = o.gmres(f, m=30, tol=1e-13, maxit=200)
    assert its > 0 and 0 < itg <= its
    for x in (xv, xg):
        assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)


def test_jacobi_cycle_differs_from_gauss_seidel_cycle(oracle_mod):
    """The smoother choice reaches the cycle: one Jacobi V-cycle is not the
    Gauss-Seidel one (a guard against the option being ignored)."""
    p = _rand_problem(15, 3, seed=4)
    f = p.rhs_paper()
    x0 = np.zeros((2 * 3 + 1) * 15 * 15)
    xj = oracle_mod.Oracle(p, theta=0.5, smoother="jacobi").vcycle(x0, f, 1)
    xg = oracle_mod.Oracle(p, theta=0.5).vcycle(x0, f, 1)
    assert np.linalg.norm(xj - xg) > 1e-3 * np.linalg.norm(xg)


def test_jacobi_counts_are_mesh_independent(oracle_mod):
    """With theta = 1/2 the V(2,2) counts stay constant as the mesh is refined,
    as Table 1 reports for the collective Jacobi smoother (row N_h), and GMRES
    needs fewer iterations than the stationary cycle."""
    counts = []
    for n in (31, 63, 127):   # at least three levels each (n_c = 7)
        p = inputs.make_problem(n, 4, 1e-4, M=6, sigma=0.5, decay=True, seed=11)
        o = oracle_mod.Oracle(p, theta=0.5, smoother="jacobi")
        _, its, _ = o.solve_vcycle(p.rhs_paper(), tol=1e-9, maxit=100)
        _, itg, _ = o.gmres(p.rhs_paper(), m=30, tol=1e-9, maxit=100)
        assert 0 < itg < its
        counts.append(its)
    assert max(counts) - min(counts) <= 2, counts
