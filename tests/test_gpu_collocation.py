"""GPU parity on stochastic-collocation instances (tensor Gauss-Hermite nodes and
weights, M = 3): non-uniform weights zeta_j in C_j and f_Y,j through the C ABI."""
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


@pytest.mark.parametrize("n,q", [(31, 3), (63, 4), (31, 5)])
def test_collocation_vcycle_iterates(B, O, n, q):
    p = inputs.collocation_problem(n, q, M=3)
    o = O.Oracle(p)
    ctx, f = B.context_from_problem(p, gmres_restart=0)
    x_o = np.zeros(o.vlen())
    xd = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    for k in range(3):
        x_o = o.vcycle(x_o, p.rhs_paper(), 1)
        ctx.vcycle(xd, f, 1)
        assert_blocks(node_to_paper(host(xd), n, p.N), x_o, n, p.N, 1e-12, k)


@pytest.mark.parametrize("n,q", [(63, 2), (63, 4)])
def test_collocation_gmres_solve(B, O, n, q):
    p = inputs.collocation_problem(n, q, M=3)
    o = O.Oracle(p)
    fp = p.rhs_paper()
    _, its_o, _ = o.gmres(fp, m=30, tol=1e-10)
    ctx, f = B.context_from_problem(p, gmres_restart=30)
    x = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    rc, st = ctx.gmres(x, f, restart=30, rtol=1e-10, maxit=100)
    assert rc == B.SMG_OK and abs(st["iterations"] - its_o) <= 1
    xg = node_to_paper(host(x), n, p.N)
    assert np.linalg.norm(o.residual(xg, fp)) <= 1e-10 * np.linalg.norm(fp)
