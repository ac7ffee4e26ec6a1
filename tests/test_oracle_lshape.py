"""Pins of the L-shaped domain (0,1)^2 minus [1/2,1)^2 of the paper's
experiments (Section 3.2), on the square grid with the removed nodes held at
zero: node counts equal to the paper's N_h, the operator equal to the
principal submatrix of the square's (the Dirichlet problem on the L-shape),
exact domains on every level, solutions and the coarsest solve equal to sparse
direct solves of the reduced system, the smoother's residual property, and
mesh-independent V-cycle counts."""
import dataclasses

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import ssn
from oracle.oracle import Oracle
from paper_2302_13680_amd import inputs


def lshape(n, N=3, nu=1e-4, seed=4, **kw):
    return inputs.make_problem(n, N, nu, M=3, sigma=0.5, decay=True, seed=seed, yd=inputs.paper_target(n), f=1.0,
                               domain="lshape", **kw)


def live_mask(p):
    """1 for the unknowns of nodes inside the domain, over all 2N+1 fields."""
    return np.tile(p.domain.ravel(), 2 * p.N + 1)


@pytest.mark.parametrize("n,nh", [(15, 161), (31, 705), (63, 2945)])
def test_node_counts_are_the_papers(n, nh):
    p = lshape(n)
    assert int(p.domain.sum()) == nh


def test_every_level_holds_the_lshape_of_its_grid():
    p = lshape(63)
    o = Oracle(p)
    for l in range(o.nlev):
        nl = o.levels_n[l]
        t = (np.arange(nl) + 1.0) / (nl + 1)
        X, Y = np.meshgrid(t, t)
        expect = (~((X >= 0.5 - 1e-12) & (Y >= 0.5 - 1e-12))).astype(float)
        np.testing.assert_array_equal(o.level_domain(l), expect)


def test_operator_is_the_principal_submatrix_of_the_square():
    p = lshape(15)
    S_sq = ssn.assemble(dataclasses.replace(p, domain=None))
    m = live_mask(p)
    o = Oracle(p)
    rng = np.random.default_rng(0)
    for _ in range(3):
        x = rng.standard_normal(m.size)
        np.testing.assert_allclose(o.apply(x), m * (S_sq @ (m * x)), rtol=1e-13, atol=1e-14)
    # and the residual has zero rows outside, whatever f holds there
    f = rng.standard_normal(m.size)
    r = o.residual(x, f)
    assert np.all(r[m == 0] == 0)


def reduced_solve(p, f):
    S_sq = ssn.assemble(dataclasses.replace(p, domain=None)).tocsr()
    idx = np.flatnonzero(live_mask(p))
    x = np.zeros(S_sq.shape[0])
    x[idx] = spla.spsolve(S_sq[idx][:, idx].tocsc(), f[idx])
    return x


@pytest.mark.parametrize("method", ["vcycle", "gmres"])
def test_solution_is_the_direct_solve_on_the_lshape(method):
    p = lshape(31, N=4)
    o = Oracle(p)
    f = p.rhs_paper()
    x_ref = reduced_solve(p, f)
    if method == "vcycle":
        x, its, _ = o.solve_vcycle(f, tol=1e-11, maxit=100)
    else:
        x, its, _ = o.gmres(f, tol=1e-11)
    assert its > 0
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-9 * np.abs(x_ref).max())


def test_red_halfsweep_solves_red_rows_and_keeps_outside_zero():
    p = lshape(15, N=5)
    o = Oracle(p)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(o.vlen())
    f = p.rhs_paper()
    xs = o.halfsweep(x, f, 0)
    r = o.residual(xs, f)
    n, N = p.n, p.N
    red = np.add.outer(np.arange(n), np.arange(n)) % 2 == 0
    live = p.domain.astype(bool)
    rows = np.tile((red & live).ravel(), 2 * N + 1)
    assert np.abs(r[rows]).max() <= 1e-12 * np.abs(r).max()
    outside_red = np.tile((red & ~live).ravel(), 2 * N + 1)
    assert np.all(xs[outside_red] == 0)


def test_coarsest_solve_is_the_direct_solve():
    p = lshape(15, N=3)
    o = Oracle(p)
    l = o.nlev - 1
    nc = o.levels_n[l]
    kx, ky = o.level_faces(l)
    c, d, e, g = o.level_scalars(l)
    q = dataclasses.replace(p, n=nc, kx=kx, ky=ky, c=c, d=d, e=e, g=g, domain=o.level_domain(l),
                            fY=np.zeros((p.N, nc, nc)), fU=np.zeros((nc, nc)), fP=np.zeros((p.N, nc, nc)))
    F = np.random.default_rng(2).standard_normal(o.vlen(l)) * live_mask(q)
    x_ref = reduced_solve(q, F)
    np.testing.assert_allclose(o.coarse_solve(F), x_ref, rtol=0, atol=1e-12 * np.abs(x_ref).max())


def test_vcycle_counts_are_mesh_independent():
    counts = []
    for n in (31, 63, 127):
        p = lshape(n, N=4)
        _, its, _ = Oracle(p).solve_vcycle(p.rhs_paper(), tol=1e-9, maxit=100)
        counts.append(its)
    assert max(counts) - min(counts) <= 2 and max(counts) <= 15, counts
