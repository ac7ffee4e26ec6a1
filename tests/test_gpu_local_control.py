"""GPU parity of local control (a per-node control mask; the paper's square-domain
experiment with the control on (0.25, 0.75)^2) against the pinned oracle,
through the C ABI: every step, cycles with both smoothers, solves in FP64 and
FP32 refinement, and the batched solver."""
import numpy as np
import pytest

from paper_2302_13680_amd import inputs
from paper_2302_13680_amd.inputs import node_to_paper, paper_to_node
from parity_util import assert_blocks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

REGION = (0.25, 0.75, 0.25, 0.75)


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


def mk(n, N, seed, region=REGION):
    return inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=seed, control_region=region)


@pytest.mark.parametrize("n,N", [(15, 3), (31, 8), (15, 100), (63, 16), (31, 256)])
def test_masked_steps(B, O, n, N):
    """Half-sweeps, residual, Jacobi step, residual + restriction on every level
    and the coarsest solve, each against the oracle with the same mask."""
    p = mk(n, N, seed=n + N)
    o = O.Oracle(p)
    ctx, _ = B.context_from_problem(p, gmres_restart=0, theta=0.5)
    rng = np.random.default_rng(n)
    x = rng.standard_normal(o.vlen())
    f = rng.standard_normal(o.vlen())
    xd, fd = dev(paper_to_node(x, n, N)), dev(paper_to_node(f, n, N))
    r = torch.empty_like(xd)
    ctx.residual(xd, fd, r)
    assert rel(node_to_paper(host(r), n, N), o.residual(x, f)) <= 1e-14
    out = torch.empty_like(xd)
    ctx.jacobi(0, xd, out, fd)
    assert rel(node_to_paper(host(out), n, N), o.jacobi(x, f, 0.5)) <= 1e-13
    xs = xd.clone()
    xo = x.copy()
    for colour in (0, 1):
        ctx.smooth(0, colour, xs, fd)
        xo = o.halfsweep(xo, f, colour, theta=0.5)
        assert rel(node_to_paper(host(xs), n, N), xo) <= 1e-13, colour
    for l in range(o.nlev - 1):
        nl, nc = o.levels_n[l], o.levels_n[l + 1]
        xl = rng.standard_normal(o.vlen(l))
        fl = rng.standard_normal(o.vlen(l))
        cd = torch.empty(o.vlen(l + 1), dtype=torch.float64, device="cuda")
        ctx.residual_restrict(l, dev(paper_to_node(xl, nl, N)), dev(paper_to_node(fl, nl, N)), cd)
        assert rel(node_to_paper(host(cd), nc, N), o.residual_restrict(xl, fl, l)) <= 1e-14, l
        cl = rng.standard_normal(o.vlen(l + 1))
        fd = dev(paper_to_node(xl, nl, N))
        ctx.prolong_add(l, dev(paper_to_node(cl, nc, N)), fd)
        assert rel(node_to_paper(host(fd), nl, N), o.prolong_control(cl, xl, l)) <= 1e-14, l
    F = rng.standard_normal(o.vlen(o.nlev - 1))
    X = torch.empty(F.size, dtype=torch.float64, device="cuda")
    nc = o.levels_n[-1]
    ctx.coarse_solve(dev(paper_to_node(F, nc, N)), X)
    assert rel(node_to_paper(host(X), nc, N), o.coarse_solve(F)) <= 1e-11


@pytest.mark.parametrize("smoother", ["gs", "jacobi"])
@pytest.mark.parametrize("n,N", [(31, 8), (63, 16), (127, 64)])
def test_masked_vcycle_iterates(B, O, smoother, n, N):
    p = mk(n, N, seed=2 * n + N)
    theta = 0.5 if smoother == "jacobi" else 1.0
    flags = B.SMG_FLAG_JACOBI if smoother == "jacobi" else 0
    o = O.Oracle(p, theta=theta, smoother=smoother)
    ctx, f = B.context_from_problem(p, gmres_restart=0, theta=theta, flags=flags)
    x_o = np.zeros(o.vlen())
    xd = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    for k in range(3):
        x_o = o.vcycle(x_o, p.rhs_paper(), 1)
        ctx.vcycle(xd, f, 1)
        assert_blocks(node_to_paper(host(xd), n, N), x_o, n, N, 1e-12, k)


@pytest.mark.parametrize("precision", [0, 1])
def test_masked_solves(B, O, precision):
    """GMRES(30) to 1e-10 (FP64; FP32 cycles in FP64 refinement): the oracle's
    residual below the tolerance and u = 0 off the control region."""
    n, N = 63, 16
    p = mk(n, N, seed=21)
    o = O.Oracle(p)
    fp = p.rhs_paper()
    ctx, f = B.context_from_problem(p, gmres_restart=30, precision=precision)
    x = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    rc, st = ctx.solve(x, f, B.SMG_GMRES, rtol=1e-10, maxit=100)
    assert rc == B.SMG_OK
    xg = node_to_paper(host(x), n, N)
    assert np.linalg.norm(o.residual(xg, fp)) <= 1e-10 * np.linalg.norm(fp)
    if precision == 0:
        _, its_o, _ = o.gmres(fp, m=30, tol=1e-10)
        assert abs(st["iterations"] - its_o) <= 1
    U = xg.reshape(2 * N + 1, n * n)[N]
    off = p.ctrl.ravel() == 0
    assert np.abs(U[off]).max() <= 1e-9 * np.abs(U).max()


def test_masked_batch_matches_single_instances(B):
    probs = [mk(63, 16, seed=31), mk(127, 32, seed=32), inputs.make_problem(63, 8, 1e-3, M=6, seed=33)]
    ctxs, xs, fs, singles = [], [], [], []
    for p in probs:
        c, f = B.context_from_problem(p, gmres_restart=0, precision=1)
        ctxs.append(c); fs.append(f)
        xs.append(torch.zeros(p.dof, dtype=torch.float64, device="cuda"))
        s, _ = B.context_from_problem(p, gmres_restart=0, precision=1)
        singles.append(s)
    bt = B.Batch(ctxs, xs, fs)
    rc, stats, _ = bt.solve(rtol=1e-8, maxit=60)
    assert rc == B.SMG_OK
    for p, s, f, xb, st in zip(probs, singles, fs, xs, stats):
        x1 = torch.zeros(p.dof, dtype=torch.float64, device="cuda")
        rc1, st1 = s.solve(x1, f, B.SMG_VCYCLE, rtol=1e-8, maxit=60)
        torch.cuda.synchronize()
        assert rc1 == B.SMG_OK and st1["iterations"] == st["iterations"]
        assert (torch.linalg.norm(x1 - xb) / torch.linalg.norm(x1)).item() <= 1e-14


def test_mask_values_outside_unit_interval_are_rejected(B):
    p = mk(15, 2, seed=3)
    bad = p.ctrl.copy()
    bad[3, 3] = 1.5
    with pytest.raises(B.SmgError) as ei:
        B.context_from_problem(p, gmres_restart=0, ctrl=bad)
    assert ei.value.code == -1
