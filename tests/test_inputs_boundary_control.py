"""Pins of the boundary-control construction (Neumann control on (0,1) x {0},
the paper's boundary-control table) against a direct discretization of the
original problem: the half-cell finite-volume system on the unit square
(half faces and half mass along Gamma, boundary mass h for the control),
assembled and solved here independently of the reflection, must give the
state, adjoint and control of the reflected system; the reflected solution is
even across the mirror row; the node counts are the paper's N_h."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import ssn
from oracle.oracle import Oracle
from paper_2302_13680_amd import inputs


@pytest.mark.parametrize("n,nh", [(31, 240), (63, 992), (127, 4032)])
def test_node_counts_are_the_papers(n, nh):
    p = inputs.boundary_control_problem(n, 2)
    mid = p.meta["mirror_row"]
    assert int(p.domain[mid:].sum()) == nh
    assert int(p.ctrl.sum()) == (n + 1) // 2 - 1


def half_domain_kkt(p):
    """The Neumann problem on the unit square assembled directly: nodes (i, r),
    x = (i+1) h, y = r h, i < m, 0 <= r <= m, Dirichlet at x = 0, 1 and y = 1;
    row r = 0 is Gamma (half cells).  Unknowns [y_1..y_N | u (Gamma) | p~_1..p~_N]."""
    n, N, h = p.n, p.N, p.meta["h"]
    mid = p.meta["mirror_row"]
    m = (n + 1) // 2 - 1
    idx = lambda i, r: r * m + i
    nh = m * (m + 1)
    zeta = p.c / (h * h)
    rows = []
    for j in range(N):
        A = sp.lil_matrix((nh, nh))
        for r in range(m + 1):
            k = mid + r                         # grid row of physical row r
            for i in range(m):
                half = 0.5 if r == 0 else 1.0
                kw, ke = p.kx[j, k, i], p.kx[j, k, i + 1]
                kn = p.ky[j, k + 1, i]
                ks = p.ky[j, k, i] if r > 0 else 0.0
                a = half * (kw + ke) + kn + ks
                A[idx(i, r), idx(i, r)] = a
                if i > 0: A[idx(i, r), idx(i - 1, r)] = -half * kw
                if i < m - 1: A[idx(i, r), idx(i + 1, r)] = -half * ke
                if r < m: A[idx(i, r), idx(i, r + 1)] = -kn
                if r > 0: A[idx(i, r), idx(i, r - 1)] = -ks
        rows.append(A.tocsr())
    mass = np.array([(0.5 if r == 0 else 1.0) * h * h for r in range(m + 1) for i in range(m)])
    gamma = np.zeros((nh, m))
    for i in range(m):
        gamma[idx(i, 0), i] = h                 # boundary mass: flux h u into the Gamma row
    Gm = sp.csr_matrix(gamma)
    yd = np.array([p.yd[mid + r, i] for r in range(m + 1) for i in range(m)])
    blocks = [[None] * (2 * N + 1) for _ in range(2 * N + 1)]
    rhs = []
    for j in range(N):
        blocks[j][j] = sp.diags(zeta[j] * mass)
        blocks[j][N + 1 + j] = rows[j].T
        blocks[N][N + 1 + j] = -Gm.T
        blocks[N + 1 + j][j] = rows[j]
        blocks[N + 1 + j][N] = -Gm
    blocks[N][N] = sp.identity(m) * (p.nu * h)
    K = sp.bmat(blocks, format="csc")
    fY = [zeta[j] * mass * yd for j in range(N)]
    f = np.concatenate(fY + [np.zeros(m)] + [np.zeros(nh)] * N)
    return spla.spsolve(K, f), m, nh


def test_reflection_equals_the_direct_neumann_discretization():
    p = inputs.boundary_control_problem(31, 3, 1e-3, seed=2)
    n, N = p.n, p.N
    nn = n * n
    mid = p.meta["mirror_row"]
    S = ssn.assemble(p, md=p.ctrl, me=p.ctrl)
    xr = spla.spsolve(S, p.rhs_paper())
    xh, m, nh = half_domain_kkt(p)
    for j in range(N):
        Yr = xr[j * nn:(j + 1) * nn].reshape(n, n)[mid:mid + m + 1, :m].ravel()
        Pr = xr[(N + 1 + j) * nn:(N + 2 + j) * nn].reshape(n, n)[mid:mid + m + 1, :m].ravel()
        Yh = xh[j * nh:(j + 1) * nh]
        Ph = xh[N * nh + m + j * nh:N * nh + m + (j + 1) * nh]
        np.testing.assert_allclose(Yr, Yh, rtol=0, atol=1e-10 * np.abs(Yh).max())
        np.testing.assert_allclose(Pr, Ph, rtol=0, atol=1e-10 * np.abs(Ph).max())
    ur = xr[N * nn:(N + 1) * nn].reshape(n, n)[mid, :m]
    uh = xh[N * nh:N * nh + m]
    np.testing.assert_allclose(ur, uh, rtol=0, atol=1e-10 * np.abs(uh).max())
    assert np.abs(uh).max() > 0


def test_reflected_solution_is_even_and_multigrid_finds_it():
    p = inputs.boundary_control_problem(63, 4, 1e-4, seed=3)
    n, N = p.n, p.N
    nn = n * n
    mid = p.meta["mirror_row"]
    o = Oracle(p)
    x, its, _ = o.gmres(p.rhs_paper(), tol=1e-11)
    assert its > 0
    Y = x[:N * nn].reshape(N, n, n)
    np.testing.assert_allclose(Y[:, :mid, :], Y[:, mid + 1:, :][:, ::-1, :], rtol=0, atol=1e-9 * np.abs(Y).max())
    U = x[N * nn:(N + 1) * nn].reshape(n, n)
    assert np.all(U[np.arange(n) != mid] == 0) and np.abs(U[mid]).max() > 0
    x_ref = spla.spsolve(ssn.assemble(p, md=p.ctrl, me=p.ctrl), p.rhs_paper())
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-8 * np.abs(x_ref).max())
