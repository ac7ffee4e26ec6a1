"""Launch modes compute the same iteration: captured hipGraph replay against
eager launches (bitwise), fused against unfused kernel sequences (rounding)."""
import numpy as np
import pytest

from paper_2302_13680_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_13680_amd import binding
    binding.load()
    return binding


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n,N", [(63, 16), (127, 64), (31, 100)])
def test_graph_replays_match_eager(B, precision, n, N):
    p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=n + N)
    ga, f = B.context_from_problem(p, gmres_restart=0, precision=precision)
    ea, _ = B.context_from_problem(p, gmres_restart=0, precision=precision, flags=B.SMG_FLAG_EAGER)
    uf, _ = B.context_from_problem(p, gmres_restart=0, precision=precision,
                                   flags=B.SMG_FLAG_EAGER | B.SMG_FLAG_UNFUSED)
    xg = torch.zeros(p.dof, dtype=torch.float64, device="cuda")
    xe = torch.zeros_like(xg)
    xu = torch.zeros_like(xg)
    for k in range(6):
        ga.vcycle(xg, f, 1)          # graph captured on the first call, replayed after
        ea.vcycle(xe, f, 1)
        uf.vcycle(xu, f, 1)
        scratch = torch.randn(1 << 20, device="cuda").sum()   # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(xg, xe), k
        rel = (torch.linalg.norm(xu - xe) / torch.linalg.norm(xe)).item()
        assert rel <= (1e-13 if precision == 0 else 1e-5), (k, rel)
        del scratch


def test_gmres_graphs_match_eager(B):
    p = inputs.make_problem(63, 32, 1e-4, M=6, sigma=0.5, decay=True, seed=3)
    ga, f = B.context_from_problem(p, gmres_restart=30)
    ea, _ = B.context_from_problem(p, gmres_restart=30, flags=B.SMG_FLAG_EAGER)
    for rep in range(3):
        xg = torch.zeros(p.dof, dtype=torch.float64, device="cuda")
        xe = torch.zeros_like(xg)
        rc1, s1 = ga.gmres(xg, f, restart=30, rtol=1e-10)
        rc2, s2 = ea.gmres(xe, f, restart=30, rtol=1e-10)
        torch.cuda.synchronize()
        assert rc1 == rc2 == 0 and s1["iterations"] == s2["iterations"]
        assert torch.equal(xg, xe), rep
