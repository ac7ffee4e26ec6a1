"""The paper's iteration-count settings on the 31x31 square (Gaussian-covariance
field, 5^3 collocation nodes, collective Jacobi theta 1/2, tolerance 1e-9):
the GPU's V-cycle and GMRES counts equal the oracle's (within one), its
solutions meet the tolerance in the oracle's residual, and the L^1 problem's
semismooth Newton run matches the oracle's Newton and inner counts."""
import numpy as np
import pytest

from paper_2302_13680_amd import inputs
from paper_2302_13680_amd.inputs import node_to_paper

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_13680_amd import binding
    binding.load()
    return binding


def paper_problem(nu, region=None, rows="scaled", domain="square"):
    return inputs.collocation_problem(31, 5, nu, M=3, sigma=float(np.sqrt(0.5)), decay=True,
                                      yd=inputs.paper_target(31), f=0.0, field="gaussian", corr_len2=0.5,
                                      control_region=region, rows=rows, domain=domain)


@pytest.mark.parametrize("region,rows,domain", [(None, "scaled", "square"), ((0.25, 0.75, 0.25, 0.75), "scaled", "square"),
                                                (None, "paper", "lshape"), ((0.25, 0.75, 0.25, 0.75), "paper", "square")])
def test_paper_setting_counts(B, region, rows, domain):
    """Both row scalings (the printed rows of eq. full_space_optimality_system
    and the symmetrized form) on the square and on the L-shape."""
    from oracle.oracle import Oracle
    p = paper_problem(1e-4, region, rows, domain)
    o = Oracle(p, smoother="jacobi", theta=0.5)
    fp = p.rhs_paper()
    ctx, f = B.context_from_problem(p, gmres_restart=30, theta=0.5, flags=B.SMG_FLAG_JACOBI)
    for method, solve in ((B.SMG_VCYCLE, lambda: o.solve_vcycle(fp, tol=1e-9, maxit=300)),
                          (B.SMG_GMRES, lambda: o.gmres(fp, tol=1e-9))):
        x = torch.zeros(p.dof, dtype=torch.float64, device="cuda")
        rc, st = ctx.solve(x, f, method, rtol=1e-9, maxit=300)
        assert rc == B.SMG_OK
        _, its, _ = solve()
        assert abs(st["iterations"] - its) <= 1, (method, st["iterations"], its)
        torch.cuda.synchronize()
        xg = node_to_paper(x.cpu().numpy(), p.n, p.N)
        assert np.linalg.norm(o.residual(xg, fp)) <= 1.01e-9 * np.linalg.norm(fp)


def test_local_control_by_galerkin_node_factors(B):
    """Local control on [0.25, 0.75]^2 as node factors of D_j and E_j coarsened by
    full weighting (the row-lumped Galerkin product), printed rows: the GPU's
    counts equal the oracle's (within one) and the solutions meet 1e-9 in the
    oracle's residual."""
    from oracle.oracle import Oracle
    p = paper_problem(1e-4, None, "paper", "square")
    t = (np.arange(p.n) + 1.0) / (p.n + 1)
    X, Y = np.meshgrid(t, t)
    m = ((X >= 0.25 - 1e-12) & (X <= 0.75 + 1e-12) & (Y >= 0.25 - 1e-12) & (Y <= 0.75 + 1e-12)).astype(np.float64)
    o = Oracle(p, smoother="jacobi", theta=0.5)
    o.set_masks(m, m, coarsen="full")
    fp = p.rhs_paper()
    ctx, f = B.context_from_problem(p, gmres_restart=30, theta=0.5, flags=B.SMG_FLAG_JACOBI)
    md = torch.tensor(m, dtype=torch.float64, device="cuda")
    ctx.set_node_factors(md, md, B.SMG_COARSEN_FULL)
    for method, solve in ((B.SMG_VCYCLE, lambda: o.solve_vcycle(fp, tol=1e-9, maxit=300)),
                          (B.SMG_GMRES, lambda: o.gmres(fp, tol=1e-9))):
        x = torch.zeros(p.dof, dtype=torch.float64, device="cuda")
        rc, st = ctx.solve(x, f, method, rtol=1e-9, maxit=300)
        assert rc == B.SMG_OK
        _, its, _ = solve()
        assert abs(st["iterations"] - its) <= 1, (method, st["iterations"], its)
        torch.cuda.synchronize()
        xg = node_to_paper(x.cpu().numpy(), p.n, p.N)
        assert np.linalg.norm(o.residual(xg, fp)) <= 1.01e-9 * np.linalg.norm(fp)


def test_paper_l1_setting(B):
    from oracle import ssn
    p = paper_problem(1e-4)
    ref = ssn.ssn_solve(p, 1e-2, -50.0, 50.0, linear="gmres", smoother="jacobi", theta=0.5)
    ctx, f = B.context_from_problem(p, gmres_restart=30, theta=0.5, flags=B.SMG_FLAG_JACOBI, ssn=True)
    x = torch.zeros(p.dof, dtype=torch.float64, device="cuda")
    prm = B.ssn_params(1e-4, 1e-2, -50.0, 50.0, (1.0 / 32) ** 2, inner_method=B.SMG_GMRES)
    rc, st = ctx.ssn_solve(x, f, prm)
    assert rc == B.SMG_OK and ref["converged"]
    assert st["iterations"] == ref["iterations"]
    assert all(abs(a - b) <= 1 for a, b in zip(st["inner"], ref["inner"]))
    nn = p.n * p.n
    ug = node_to_paper(x.cpu().numpy(), p.n, p.N)[p.N * nn:(p.N + 1) * nn]
    assert np.abs(ug - ref["u"]).max() <= 1e-8 * np.abs(ref["u"]).max()
