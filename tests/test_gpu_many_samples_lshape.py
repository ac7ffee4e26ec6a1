"""GPU parity of the many-sample kernels (256-lane groups above 512 samples) in
the setting of the paper's Monte Carlo sub-tables: the L-shape, damped
collective Jacobi (theta 1/2), N = 777 and 2000.  The Jacobi step and the
prolongation on the two finest levels, V-cycle iterates in FP64 and FP32 per
block, and a risk-averse solve above 512 samples checked by the oracle's
F_1 and F_2."""
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


def problem(N, n=31, seed=1):
    return inputs.make_problem(n, N, 1e-4, M=15, sigma=float(np.sqrt(1.5)), decay=True, seed=seed,
                               field="gaussian", corr_len2=0.1, yd=inputs.paper_target(n), f=0.0,
                               domain="lshape")


def live(o, N, l):
    return np.tile(o.level_domain(l).ravel(), 2 * N + 1)


@pytest.mark.parametrize("N", [777, 2000])
def test_jacobi_and_prolongation_on_two_levels(B, O, N):
    p = problem(N, seed=N)
    o = O.Oracle(p, theta=0.5, smoother="jacobi")
    ctx, _ = B.context_from_problem(p, gmres_restart=0, theta=0.5, flags=B.SMG_FLAG_JACOBI)
    rng = np.random.default_rng(N)
    for l in (0, 1):
        nl, nc = o.levels_n[l], o.levels_n[l + 1]
        x = rng.standard_normal(o.vlen(l)) * live(o, N, l)
        f = rng.standard_normal(o.vlen(l))
        xd, fd = dev(paper_to_node(x, nl, N)), dev(paper_to_node(f, nl, N))
        out = torch.empty_like(xd)
        ctx.jacobi(l, xd, out, fd)
        assert_blocks(node_to_paper(host(out), nl, N), o.jacobi(x, f, 0.5, l), nl, N, 1e-13, ("jacobi", l))
        cl = rng.standard_normal(o.vlen(l + 1)) * live(o, N, l + 1)
        fine = xd.clone()
        ctx.prolong_add(l, dev(paper_to_node(cl, nc, N)), fine)
        assert_blocks(node_to_paper(host(fine), nl, N), o.prolong_control(cl, x, l), nl, N, 1e-15,
                      ("prolong", l))


@pytest.mark.parametrize("N", [777, 2000])
@pytest.mark.parametrize("precision", [0, 1])
def test_jacobi_vcycle_iterates(B, O, N, precision):
    p = problem(N)
    o = O.Oracle(p, theta=0.5, smoother="jacobi")
    ctx, f = B.context_from_problem(p, gmres_restart=0, theta=0.5, flags=B.SMG_FLAG_JACOBI, precision=precision)
    fp = p.rhs_paper()
    x_o = np.zeros(o.vlen())
    xd = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    cyc = o.vcycle if precision == 0 else o.vcycle32
    for k in range(2):
        x_o = cyc(x_o, fp, 1)
        ctx.vcycle(xd, f, 1)
        assert_blocks(node_to_paper(host(xd), p.n, N), x_o, p.n, N, 1e-12 if precision == 0 else 2e-5, k)


def test_cvar_above_512_samples(B):
    """The risk-averse table's problem at N = 1000 (lambda 0.95, eps 1e-2): the
    GPU's result zeroes F_1 and F_2 in the oracle's arithmetic."""
    from oracle import cvar as cv
    p = inputs.make_problem(31, 1000, 1e-4, M=15, sigma=1.0, seed=23, yd=inputs.paper_target(31), f=0.0,
                            field="gaussian", corr_len2=0.1, domain="lshape")
    c = cv.Cvar(p, 0.95, 1e-2)
    ctx, f = B.context_from_problem(p, gmres_restart=30, theta=0.5, flags=B.SMG_FLAG_JACOBI | B.SMG_FLAG_CVAR)
    x = torch.zeros(c.o.vlen(), dtype=torch.float64, device="cuda")
    yd = torch.tensor(c.yd.reshape(p.n, p.n), dtype=torch.float64, device="cuda")
    rc, st = ctx.cvar_solve(x, f, yd, c.zeta, 0.95, 1e-2, c.mass)
    assert rc == B.SMG_OK and 1 <= st["outer"] <= 10
    xg = node_to_paper(host(x), p.n, p.N)
    z, q = c.z_q(xg)
    assert abs(c.F4(q, st["t"])) <= 1e-6
    F1 = c.F1(xg, st["t"])
    assert np.linalg.norm(F1) <= 1e-8 * max(1.0, np.linalg.norm(c.rhs(c.c_of(q, st["t"]))))
    assert abs(np.sum(c.zeta * cv.dg_eps(q - st["t"], 1e-2)) - 0.05) <= 1e-6
    ctx.close()
