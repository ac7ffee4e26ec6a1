"""smg_residual_static, the residual entry point that allocates nothing (its
partial sums in the library's static device scratch, its norms to a device
buffer), against smg_residual (the context's workspace): two calls in a row on
one GPU, the second on a smaller grid, bitwise equal residuals and norms, the
norms confirmed by the oracle; replays of a captured graph; the size limit."""
import numpy as np
import pytest

from paper_2302_13680_amd import inputs
from paper_2302_13680_amd.inputs import node_to_paper, paper_to_node

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_13680_amd import binding
    binding.load()
    return binding


def test_static_residual_equals_workspace_residual_twice(B):
    from oracle import oracle as O
    for n, N, seed in ((255, 64, 1), (63, 16, 2)):          # the second call on a smaller grid
        p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=seed)
        ctx, f = B.context_from_problem(p, gmres_restart=0)
        rng = np.random.default_rng(seed)
        xh = rng.standard_normal(p.dof)
        x = torch.from_numpy(paper_to_node(xh, n, N)).cuda()
        r1 = torch.empty_like(x)
        h = ctx.residual(x, f, r1, norms=True)
        r2 = torch.full_like(x, float("nan"))
        nd = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.residual_static(x, f, r2, nd)
        torch.cuda.synchronize()
        assert torch.equal(r1, r2), (n, N)
        got = nd.cpu().numpy()
        assert np.array_equal(got[:4], np.array(h)), (got, h)
        fp = p.rhs_paper()
        assert got[4] == pytest.approx(np.linalg.norm(fp), rel=1e-14)
        ro = O.Oracle(p).residual(xh, fp)
        assert np.linalg.norm(node_to_paper(r2.cpu().numpy(), n, N) - ro) <= 1e-14 * np.linalg.norm(ro)
        assert got[0] == pytest.approx(np.linalg.norm(ro), rel=1e-13)
        ctx.close()


def test_static_residual_in_a_captured_graph(B):
    """Captured once, replayed three times with eager work and synchronizations
    between the replays; every replay equals the eager call."""
    p = inputs.make_problem(127, 32, 1e-4, M=6, sigma=0.5, decay=True, seed=3)
    s = torch.cuda.Stream()
    ctx, f = B.context_from_problem(p, gmres_restart=0, stream=s)
    x = torch.rand(p.dof, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    torch.cuda.synchronize()
    r_ref = torch.empty_like(x)
    n_ref = torch.empty(5, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(s):
        ctx.residual_static(x, f, r_ref, n_ref)
    s.synchronize()
    r = torch.zeros_like(x)
    nd = torch.zeros(5, dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ctx.residual_static(x, f, r, nd)
    for rep in range(3):
        r.zero_()
        nd.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(r, r_ref) and torch.equal(nd, n_ref), rep
        ctx.apply(x, r)                      # eager work on the same stream between replays
        torch.cuda.synchronize()
    ctx.close()


def test_static_residual_rejects_grids_beyond_its_scratch(B):
    """2047 x 2047 nodes with 64 lanes per node needs 4.2e6 doubles of partial
    sums, more than the 1.05e6 the library holds: SMG_EWORKSPACE, nothing
    launched (the context's own smg_residual still works)."""
    n, N = 2047, 33
    kx = torch.ones((n, n + 1, N), dtype=torch.float64, device="cuda")
    ky = torch.ones((n + 1, n, N), dtype=torch.float64, device="cuda")
    h2 = (1.0 / (n + 1)) ** 2
    ctx = B.Context(n, N, kx, ky, [h2 / N] * N, [-h2] * N, [-h2] * N, 1e-4 * h2, gmres_restart=0)
    x = torch.zeros(ctx.vlen(), dtype=torch.float64, device="cuda")
    f = torch.ones_like(x)
    r = torch.empty_like(x)
    nd = torch.zeros(5, dtype=torch.float64, device="cuda")
    with pytest.raises(B.SmgError) as ei:
        ctx.residual_static(x, f, r, nd)
    assert ei.value.code == -5 and "scratch" in str(ei.value)
    h = ctx.residual(x, f, r, norms=True)
    assert h[0] == pytest.approx(np.sqrt(float(ctx.vlen())), rel=1e-12)
    ctx.close()
