"""Batched solves of uneven instances: one graph launch per refinement step for
all instances, device-side retirement.  Checked against the oracle (counts,
residuals) and against the single-instance path, whose per-node arithmetic is
the same device code."""
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


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as o
    return o


SPECS = [(31, 8, 1e-4, 101), (63, 16, 1e-6, 102), (127, 32, 1e-2, 103), (63, 100, 1e-5, 104),
         (31, 64, 1e-3, 105), (127, 16, 1e-4, 106), (15, 4, 1e-4, 107)]


def _problems():
    return [inputs.make_problem(n, N, nu, M=6, sigma=0.5, decay=True, seed=s) for (n, N, nu, s) in SPECS]


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_against_oracle(B, O, precision):
    probs = _problems()
    ctxs, xs, fs = [], [], []
    for p in probs:
        c, f = B.context_from_problem(p, gmres_restart=0, precision=precision)
        ctxs.append(c); fs.append(f)
        xs.append(torch.zeros(p.dof, dtype=torch.float64, device="cuda"))
    bt = B.Batch(ctxs, xs, fs)
    for rep in range(2):                        # graph captured once, replayed
        for x in xs:
            x.zero_()
        rc, stats, wall = bt.solve(rtol=1e-8, maxit=60)
        assert rc == B.SMG_OK
        torch.cuda.synchronize()
        for p, x, st in zip(probs, xs, stats):
            o = O.Oracle(p)
            fp = p.rhs_paper()
            xg = node_to_paper(x.cpu().numpy(), p.n, p.N)
            assert np.linalg.norm(o.residual(xg, fp)) <= 1e-8 * np.linalg.norm(fp)
            if precision == 0:
                _, its, _ = o.solve_vcycle(fp, tol=1e-8)
            else:
                _, its, _, _ = o.solve_ir(fp, tol=1e-8, m=0)
            assert abs(st["iterations"] - its) <= 1, (p.n, p.N, st["iterations"], its)
            assert st["relres"] <= 1e-8
            assert st["time_ms"] > 0


def test_batch_equals_single_instance_refinement(B):
    """With the default lane widths the batched kernels run the same per-node
    arithmetic as the single-instance FP32 refinement: the same refinement
    counts and iterates equal to rounding.  (The FP64 refinement residual takes
    two samples per access in the batch wherever every N is even, and the
    single-instance kernel only with 64 lanes per node, so for small N the sum
    over samples in the control row runs in another order: 2.6e-14 observed.)"""
    probs = _problems()
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
        assert rc1 == B.SMG_OK
        assert st1["iterations"] == st["iterations"]
        rel = (torch.linalg.norm(x1 - xb) / torch.linalg.norm(x1)).item()
        assert rel <= 1e-13, (p.n, p.N, rel)


def test_autotuned_lanes(B, O, tmp_path):
    from paper_2302_13680_amd import autotune
    probs = _problems()[:4]
    ctxs, xs, fs = [], [], []
    for p in probs:
        c, f = B.context_from_problem(p, gmres_restart=0, precision=1)
        ctxs.append(c); fs.append(f)
        xs.append(torch.zeros(p.dof, dtype=torch.float64, device="cuda"))
    cache = str(tmp_path / "tune.json")
    lanes, table = autotune.tune(ctxs, cache)
    for p, w in zip(probs, lanes):
        assert w in (1, 2, 4, 8, 16, 32, 64) and (p.N + w - 1) // w <= 8
    # the batch-wide samples per lane stay at the smallest value the batch allows
    # (two samples per access: FP32 with every N even)
    v = 2 if all(p.N % 2 == 0 for p in probs) else 1
    jm = lambda N, w: v * -(-N // (v * w))
    assert max(jm(p.N, w) for p, w in zip(probs, lanes)) == max(jm(p.N, 64) for p in probs)
    lanes2, _ = autotune.tune(ctxs, cache)          # served from the cache
    assert lanes2 == lanes
    bt = B.Batch(ctxs, xs, fs, lanes=lanes)
    rc, stats, _ = bt.solve(rtol=1e-8, maxit=60)
    assert rc == B.SMG_OK
    torch.cuda.synchronize()
    for p, x in zip(probs, xs):
        o = O.Oracle(p)
        fp = p.rhs_paper()
        xg = node_to_paper(x.cpu().numpy(), p.n, p.N)
        assert np.linalg.norm(o.residual(xg, fp)) <= 1e-8 * np.linalg.norm(fp)


def test_batch_iteration_limit(B):
    probs = _problems()[:3]
    ctxs, xs, fs = [], [], []
    for p in probs:
        c, f = B.context_from_problem(p, gmres_restart=0, precision=1)
        ctxs.append(c); fs.append(f)
        xs.append(torch.zeros(p.dof, dtype=torch.float64, device="cuda"))
    bt = B.Batch(ctxs, xs, fs)
    rc, stats, _ = bt.solve(rtol=1e-12, maxit=2)
    assert rc == B.SMG_NOT_CONVERGED
    assert all(st["iterations"] == 2 for st in stats)


def test_batch_with_the_largest_instances(B, O):
    """The extremes of the uneven workload in one batch: 255x255 with N = 128 and
    with N = 16, 63x63 with N = 128 and N = 16, nu from 1e-6 to 1e-2, in the
    FP32-refined form; every instance meets 1e-8 by the oracle's FP64 residual
    with the oracle's refinement count within one."""
    specs = [(255, 128, 1e-6, 201), (63, 16, 1e-2, 202), (255, 16, 1e-4, 203), (63, 128, 1e-3, 204)]
    probs = [inputs.make_problem(n, N, nu, M=6, sigma=0.5, decay=True, seed=s) for (n, N, nu, s) in specs]
    ctxs, xs, fs = [], [], []
    for p in probs:
        c, f = B.context_from_problem(p, gmres_restart=0, precision=1)
        ctxs.append(c); fs.append(f)
        xs.append(torch.zeros(p.dof, dtype=torch.float64, device="cuda"))
    bt = B.Batch(ctxs, xs, fs)
    rc, stats, _ = bt.solve(rtol=1e-8, maxit=60)
    assert rc == B.SMG_OK
    torch.cuda.synchronize()
    for p, x, st in zip(probs, xs, stats):
        o = O.Oracle(p)
        fp = p.rhs_paper()
        xg = node_to_paper(x.cpu().numpy(), p.n, p.N)
        assert np.linalg.norm(o.residual(xg, fp)) <= 1e-8 * np.linalg.norm(fp), (p.n, p.N)
        _, its, _, _ = o.solve_ir(fp, tol=1e-8, m=0)
        assert abs(st["iterations"] - its) <= 1, (p.n, p.N, st["iterations"], its)
