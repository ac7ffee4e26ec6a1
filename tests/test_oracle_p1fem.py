"""Pins of the P1 / Galerkin model of the paper's experiments (oracle/p1fem.py):
element matrices against their closed forms on the right-triangle mesh, the
Galerkin products against the coarse mesh's own matrices (nested P1 spaces),
the closed-form node solve against dense solves of the node blocks, and the
V-cycle and GMRES against a sparse direct solve."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import p1fem


def _grid_neighbours(mesh, r):
    i, k = mesh.nodes[r]
    out = {}
    for name, (di, dk) in dict(W=(-1, 0), E=(1, 0), S=(0, -1), N=(0, 1), SW=(-1, -1), NE=(1, 1),
                               NW=(-1, 1), SE=(1, -1)).items():
        c = mesh.idx[k + dk, i + di]
        if c >= 0:
            out[name] = c
    return out


def test_stiffness_and_mass_closed_forms():
    mesh = p1fem.Mesh(16)
    K = mesh.stiffness(np.ones(len(mesh.tris))).toarray()
    Mm = mesh.mass().toarray()
    h2 = mesh.h ** 2
    for r in range(mesh.n):
        nb = _grid_neighbours(mesh, r)
        assert np.isclose(K[r, r], 4.0)                  # every interior node has six triangles
        for name, c in nb.items():
            want = -1.0 if name in ("W", "E", "S", "N") else 0.0   # no coupling across a hypotenuse
            assert np.isclose(K[r, c], want, atol=1e-14), (r, name)
        assert np.isclose(Mm[r, r], h2 / 2)             # 6 triangles x (h^2/2)/6
        for name, c in nb.items():
            want = h2 / 12 if name in ("W", "E", "S", "N", "SW", "NE") else 0.0
            assert np.isclose(Mm[r, c], want, atol=1e-16), (r, name)
    assert mesh.n == 161
    assert p1fem.Mesh(32).n == 705 and p1fem.Mesh(64).n == 2945   # the paper's N_h


def test_galerkin_products_equal_the_coarse_mesh_matrices():
    fine, coarse = p1fem.Mesh(32), p1fem.Mesh(16)
    P = p1fem.prolongation(coarse, fine)
    Kf = fine.stiffness(np.ones(len(fine.tris)))
    Kc = coarse.stiffness(np.ones(len(coarse.tris)))
    assert abs(P.T @ Kf @ P - Kc).max() <= 1e-12
    assert abs(P.T @ fine.mass() @ P - coarse.mass()).max() <= 1e-16
    # P reproduces linear functions on the unknowns away from the boundary
    xc = coarse.nodes[:, 0] * coarse.h
    xf = fine.nodes[:, 0] * fine.h
    inner = np.array([np.all([fine.idx[k + dk, i + di] >= 0 for di in (-1, 0, 1) for dk in (-1, 0, 1)])
                      for i, k in fine.nodes])
    assert np.allclose((P @ xc)[inner], xf[inner])


def test_node_solve_against_dense_node_blocks():
    H, f = p1fem.table1_problem(m_fine=16, q=2, nu=1e-3)
    L = H.levels[0]
    rng = np.random.default_rng(0)
    r = rng.standard_normal(f.size)
    got = L.node_solve(r)
    S = L.assemble().tocsr()
    N, n = L.N, L.n
    for i in (0, 17, n - 1):
        idx = [j * n + i for j in range(N)] + [N * n + i] + [(N + 1) * n + j * n + i for j in range(N)]
        D = S[idx][:, idx].toarray()                    # eq. reduced_matrices at node i
        assert np.count_nonzero(D[:N, :N] - np.diag(np.diag(D[:N, :N]))) == 0
        assert np.allclose(got[idx], np.linalg.solve(D, r[idx]), rtol=1e-12, atol=1e-14)


def test_vcycle_and_gmres_reach_the_direct_solution():
    H, f = p1fem.table1_problem(m_fine=16, q=2, nu=1e-3)
    xs = spla.spsolve(H.levels[0].assemble(), f)
    xv, kv = H.solve_vcycle(f, tol=1e-10)
    xg, kg = H.gmres(f, tol=1e-10)
    assert 0 < kv < 60 and 0 < kg < 30
    for x in (xv, xg):
        assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
