"""GPU parity of Neumann boundary control (the reflected system: a domain and a
control on the mirror row) against the oracle: V-cycle iterates, solves with
both smoothers, and the paper's boundary-control setting."""
import numpy as np
import pytest

from paper_2302_13680_amd import inputs
from paper_2302_13680_amd.inputs import node_to_paper
from parity_util import assert_blocks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_13680_amd import binding
    binding.load()
    return binding


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as o
    return o


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("smoother", ["gs", "jacobi"])
def test_boundary_control_cycles_and_solves(B, O, smoother):
    n, N = 63, 8
    p = inputs.boundary_control_problem(n, N, 1e-4, seed=5)
    theta = 0.5 if smoother == "jacobi" else 1.0
    flags = B.SMG_FLAG_JACOBI if smoother == "jacobi" else 0
    o = O.Oracle(p, smoother=smoother, theta=theta)
    ctx, f = B.context_from_problem(p, gmres_restart=30, theta=theta, flags=flags)
    fp = p.rhs_paper()
    x_o = np.zeros(o.vlen())
    xd = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    for k in range(3):
        x_o = o.vcycle(x_o, fp, 1)
        ctx.vcycle(xd, f, 1)
        assert_blocks(node_to_paper(host(xd), n, N), x_o, n, N, 1e-12, k)
    for method, solve in ((B.SMG_VCYCLE, lambda: o.solve_vcycle(fp, tol=1e-9, maxit=300)),
                          (B.SMG_GMRES, lambda: o.gmres(fp, tol=1e-9))):
        xd.zero_()
        rc, st = ctx.solve(xd, f, method, rtol=1e-9, maxit=300)
        assert rc == B.SMG_OK
        _, its, _ = solve()
        assert abs(st["iterations"] - its) <= 1
        xg = node_to_paper(host(xd), n, N)
        assert np.linalg.norm(o.residual(xg, fp)) <= 1.01e-9 * np.linalg.norm(fp)
        U = xg[N * n * n:(N + 1) * n * n].reshape(n, n)
        mid = p.meta["mirror_row"]
        # u off Gamma is outside the control space: no correction ever reaches it
        assert np.abs(U[np.arange(n) != mid]).max() == 0


def test_boundary_control_paper_setting(B, O):
    """31x32 physical nodes (N_h = 992), the Gaussian field, 5^3 collocation
    nodes, Jacobi theta 1/2, tolerance 1e-9: GPU and oracle counts agree."""
    p = inputs.boundary_collocation_problem(63, 5, 1e-4, sigma=float(np.sqrt(0.5)), field="gaussian",
                                            corr_len2=0.5)
    o = O.Oracle(p, smoother="jacobi", theta=0.5)
    ctx, f = B.context_from_problem(p, gmres_restart=30, theta=0.5, flags=B.SMG_FLAG_JACOBI)
    fp = p.rhs_paper()
    for method, solve in ((B.SMG_VCYCLE, lambda: o.solve_vcycle(fp, tol=1e-9, maxit=300)),
                          (B.SMG_GMRES, lambda: o.gmres(fp, tol=1e-9))):
        x = torch.zeros(p.dof, dtype=torch.float64, device="cuda")
        rc, st = ctx.solve(x, f, method, rtol=1e-9, maxit=300)
        assert rc == B.SMG_OK
        _, its, _ = solve()
        assert abs(st["iterations"] - its) <= 1
