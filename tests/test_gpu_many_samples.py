"""GPU parity with many samples (N = 1000 and 2000, the paper's Monte Carlo
sub-tables: 64 lanes per node with 16 or 32 samples each) against the oracle:
every step, V-cycle iterates in FP64 and FP32, and solves."""
import numpy as np
import pytest

from paper_2302_13680_amd import inputs
from paper_2302_13680_amd.inputs import node_to_paper, paper_to_node
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("N", [1000, 2000, 777])
def test_many_sample_steps(B, O, N):
    n = 15
    p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=N)
    o = O.Oracle(p, theta=0.5)
    ctx, _ = B.context_from_problem(p, gmres_restart=0, theta=0.5)
    rng = np.random.default_rng(N)
    x = rng.standard_normal(o.vlen())
    f = rng.standard_normal(o.vlen())
    xd, fd = dev(paper_to_node(x, n, N)), dev(paper_to_node(f, n, N))
    r = torch.empty_like(xd)
    ctx.residual(xd, fd, r)
    assert rel(node_to_paper(host(r), n, N), o.residual(x, f)) <= 1e-14
    out = torch.empty_like(xd)
    ctx.jacobi(0, xd, out, fd)
    assert rel(node_to_paper(host(out), n, N), o.jacobi(x, f, 0.5)) <= 1e-13
    xs, xo = xd.clone(), x.copy()
    for colour in (0, 1):
        ctx.smooth(0, colour, xs, fd)
        xo = o.halfsweep(xo, f, colour, theta=0.5)
        assert rel(node_to_paper(host(xs), n, N), xo) <= 1e-13, colour
    nc = o.levels_n[1]
    cd = torch.empty(o.vlen(1), dtype=torch.float64, device="cuda")
    ctx.residual_restrict(0, xd, fd, cd)
    assert rel(node_to_paper(host(cd), nc, N), O.restrict(n, N, o.residual(x, f))) <= 1e-14
    cl = rng.standard_normal(o.vlen(1))
    fine = xd.clone()
    ctx.prolong_add(0, dev(paper_to_node(cl, nc, N)), fine)
    assert rel(node_to_paper(host(fine), n, N), O.prolong_add(nc, N, cl, x)) <= 1e-15
    F = rng.standard_normal(o.vlen(1))
    X = torch.empty(F.size, dtype=torch.float64, device="cuda")
    ctx.coarse_solve(dev(paper_to_node(F, nc, N)), X)
    assert rel(node_to_paper(host(X), nc, N), o.coarse_solve(F)) <= 1e-11


@pytest.mark.parametrize("precision", [0, 1])
def test_many_sample_cycles_and_solve(B, O, precision):
    n, N = 31, 2000
    p = inputs.make_problem(n, N, 1e-4, M=15, sigma=float(np.sqrt(1.5)), decay=True, seed=1, field="gaussian",
                            corr_len2=0.1, yd=inputs.paper_target(n), f=0.0, domain="lshape")
    o = O.Oracle(p)
    ctx, f = B.context_from_problem(p, gmres_restart=30, precision=precision)
    fp = p.rhs_paper()
    x_o = np.zeros(o.vlen())
    xd = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    cyc = o.vcycle if precision == 0 else o.vcycle32
    for k in range(2):
        x_o = cyc(x_o, fp, 1)
        ctx.vcycle(xd, f, 1)
        assert_blocks(node_to_paper(host(xd), n, N), x_o, n, N, 1e-12 if precision == 0 else 2e-5, k)
    xd.zero_()
    rc, st = ctx.solve(xd, f, B.SMG_GMRES, rtol=1e-9, maxit=100)
    assert rc == B.SMG_OK
    xg = node_to_paper(host(xd), n, N)
    assert np.linalg.norm(o.residual(xg, fp)) <= 1.01e-9 * np.linalg.norm(fp)
    if precision == 0:
        _, its, _ = o.gmres(fp, tol=1e-9)
        assert abs(st["iterations"] - its) <= 1
