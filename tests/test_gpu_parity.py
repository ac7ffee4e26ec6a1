"""GPU parity: every step of the HIP path against the CPU oracle, through the C ABI.

Tolerances (FP64): elementwise steps agree to 1e-13 relative (only the
rounding order differs: FMA contraction, tree vs serial sums over samples);
iterates after k V-cycles to 1e-12 relative; solves reach ||f - S x|| <=
1e-10 ||f|| evaluated by the oracle, with the same iteration counts (+-1 for
GMRES, whose orthogonalization differs: CGS2 against MGS).
"""
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


def mk(n, N, seed=0, nu=1e-4, sigma=0.5, M=4, decay=False):
    return inputs.make_problem(n, N, nu, M=M, sigma=sigma, decay=decay, seed=seed)


SMALL = [(15, 1), (15, 3), (31, 8), (15, 33), (15, 64), (15, 100), (7, 256), (63, 16), (15, 300), (7, 512)]


@pytest.mark.parametrize("n,N", SMALL)
def test_apply_and_residual(B, O, n, N):
    p = mk(n, N, seed=n + N)
    o = O.Oracle(p, coarsest_n=7 if n >= 7 else 1)
    ctx, f = B.context_from_problem(p, gmres_restart=0)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(o.vlen())
    ref = o.apply(x)
    out = torch.empty(o.vlen(), dtype=torch.float64, device="cuda")
    ctx.apply(dev(paper_to_node(x, n, N)), out)
    got = node_to_paper(host(out), n, N)
    assert rel(got, ref) <= 1e-14
    r = torch.empty_like(out)
    norms = ctx.residual(dev(paper_to_node(x, n, N)), f, r, norms=True)
    rref = o.residual(x, p.rhs_paper())
    assert rel(node_to_paper(host(r), n, N), rref) <= 1e-14
    nn = n * n
    assert abs(norms[0] - np.linalg.norm(rref)) <= 1e-13 * np.linalg.norm(rref)
    assert abs(norms[1] - np.linalg.norm(rref[:N * nn])) <= 1e-13 * np.linalg.norm(rref)
    assert abs(norms[2] - np.linalg.norm(rref[N * nn:(N + 1) * nn])) <= 1e-13 * np.linalg.norm(rref)
    assert abs(norms[3] - np.linalg.norm(rref[(N + 1) * nn:])) <= 1e-13 * np.linalg.norm(rref)


@pytest.mark.parametrize("n,N", SMALL)
@pytest.mark.parametrize("theta", [1.0, 0.7])
def test_halfsweeps(B, O, n, N, theta):
    p = mk(n, N, seed=2 * n + N)
    o = O.Oracle(p, coarsest_n=7, theta=theta)
    ctx, f = B.context_from_problem(p, gmres_restart=0, theta=theta)
    x = np.random.default_rng(3).standard_normal(o.vlen())
    fp = p.rhs_paper()
    xd = dev(paper_to_node(x, n, N))
    for colour in (0, 1, 0, 1):
        x = o.halfsweep(x, fp, colour, theta=theta)
        ctx.smooth(0, colour, xd, f)
        assert rel(node_to_paper(host(xd), n, N), x) <= 1e-13, colour


@pytest.mark.parametrize("n,N", [(63, 16), (31, 100), (127, 64)])
@pytest.mark.parametrize("strip", [2, 8, 30])
def test_halfsweeps_strip_order(B, O, n, N, strip):
    """The strip traversal visits the nodes of a colour in another order; a
    half-sweep reads only the other colour, so the iterates are bitwise those of
    row-major order, and match the oracle."""
    p = mk(n, N, seed=n + strip)
    o = O.Oracle(p, coarsest_n=7)
    c_row, f = B.context_from_problem(p, gmres_restart=0, strip=n + 1)
    c_str, _ = B.context_from_problem(p, gmres_restart=0, strip=strip)
    x = np.random.default_rng(4).standard_normal(o.vlen())
    fp = p.rhs_paper()
    xa, xb = dev(paper_to_node(x, n, N)), dev(paper_to_node(x, n, N))
    for colour in (0, 1, 0, 1):
        x = o.halfsweep(x, fp, colour)
        c_row.smooth(0, colour, xa, f)
        c_str.smooth(0, colour, xb, f)
        assert torch.equal(xa, xb), colour
        assert rel(node_to_paper(host(xb), n, N), x) <= 1e-13, colour


@pytest.mark.parametrize("n,N", [(31, 8), (63, 16), (31, 100)])
def test_hierarchy_faces_bit_exact(B, O, n, N):
    p = mk(n, N, seed=5)
    o = O.Oracle(p)
    ctx, _ = B.context_from_problem(p, gmres_restart=0)
    assert ctx.levels_n == o.levels_n
    for l in range(1, o.nlev):
        kx_o, ky_o = o.level_faces(l)
        nl = o.levels_n[l]
        kx = torch.empty(nl * (nl + 1) * N, dtype=torch.float64, device="cuda")
        ky = torch.empty_like(kx)
        ctx.level_faces(l, kx, ky)
        np.testing.assert_array_equal(host(kx).reshape(nl, nl + 1, N).transpose(2, 0, 1), kx_o)
        np.testing.assert_array_equal(host(ky).reshape(nl + 1, nl, N).transpose(2, 0, 1), ky_o)


@pytest.mark.parametrize("n,N", [(31, 8), (63, 3), (31, 100)])
def test_transfers(B, O, n, N):
    p = mk(n, N, seed=6)
    ctx, _ = B.context_from_problem(p, gmres_restart=0)
    nc = (n - 1) // 2
    rng = np.random.default_rng(7)
    fine = rng.standard_normal((2 * N + 1) * n * n)
    coarse = rng.standard_normal((2 * N + 1) * nc * nc)
    cd = torch.empty(coarse.size, dtype=torch.float64, device="cuda")
    ctx.restrict(0, dev(paper_to_node(fine, n, N)), cd)
    assert rel(node_to_paper(host(cd), nc, N), O.restrict(n, N, fine)) <= 1e-15
    fd = dev(paper_to_node(fine, n, N))
    ctx.prolong_add(0, dev(paper_to_node(coarse, nc, N)), fd)
    assert rel(node_to_paper(host(fd), n, N), O.prolong_add(nc, N, coarse, fine)) <= 1e-15


@pytest.mark.parametrize("n,N", [(15, 1), (15, 3), (31, 8), (15, 33), (15, 64), (63, 16), (15, 100),
                                 (15, 300), (31, 256)])
def test_residual_restrict(B, O, n, N):
    # one pass R (f - S x) on every level with a coarser one: against the
    # oracle's residual then restriction, and against the two GPU passes (the
    # control row sums over samples once instead of per fine node: rounding)
    p = mk(n, N, seed=n + 2 * N)
    o = O.Oracle(p)
    ctx, _ = B.context_from_problem(p, gmres_restart=0)
    rng = np.random.default_rng(n * N)
    for l in range(o.nlev - 1):
        nl = o.levels_n[l]
        nc = o.levels_n[l + 1]
        x = rng.standard_normal((2 * N + 1) * nl * nl)
        f = rng.standard_normal(x.size)
        cd = torch.empty((2 * N + 1) * nc * nc, dtype=torch.float64, device="cuda")
        ctx.residual_restrict(l, dev(paper_to_node(x, nl, N)), dev(paper_to_node(f, nl, N)), cd)
        ref = O.restrict(nl, N, o.residual(x, f, l))
        assert rel(node_to_paper(host(cd), nc, N), ref) <= 1e-14, l
        if l == 0:
            r = torch.empty(x.size, dtype=torch.float64, device="cuda")
            c2 = torch.empty_like(cd)
            ctx.residual(dev(paper_to_node(x, nl, N)), dev(paper_to_node(f, nl, N)), r)
            ctx.restrict(0, r, c2)
            assert rel(host(cd), host(c2)) <= 1e-15


@pytest.mark.parametrize("N", [1, 5, 64, 300, 512])
def test_coarse_solve(B, O, N):
    p = mk(7, N, seed=8)
    o = O.Oracle(p, coarsest_n=7)
    ctx, _ = B.context_from_problem(p, gmres_restart=0)
    F = np.random.default_rng(9).standard_normal(o.vlen())
    X = torch.empty(o.vlen(), dtype=torch.float64, device="cuda")
    ctx.coarse_solve(dev(paper_to_node(F, 7, N)), X)
    assert rel(node_to_paper(host(X), 7, N), o.coarse_solve(F)) <= 1e-11


CYCLE_CASES = [(31, 8, 0), (63, 16, 1), (127, 64, 2), (15, 1, 3), (31, 100, 4), (7, 4, 5)]


@pytest.mark.parametrize("n,N,seed", CYCLE_CASES)
def test_vcycle_iterates(B, O, n, N, seed):
    """k = 1..5 cycles from zero with the same sweep order agree to 1e-12."""
    p = mk(n, N, seed=seed, M=6, decay=True)
    o = O.Oracle(p)
    ctx, f = B.context_from_problem(p, gmres_restart=0)
    x_o = np.zeros(o.vlen())
    xd = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    for k in range(5):
        x_o = o.vcycle(x_o, p.rhs_paper(), 1)
        ctx.vcycle(xd, f, 1)
        assert_blocks(node_to_paper(host(xd), n, N), x_o, n, N, 1e-12, k)


def test_small_problem_stationary_solve(B, O):
    """31x31, N = 8, nu = 1e-4: V(2,2) to 1e-10, same count as the oracle, and the
    oracle confirms the residual of the GPU solution."""
    p = inputs.small_fp64()
    o = O.Oracle(p)
    x_o, its_o, _ = o.solve_vcycle(p.rhs_paper(), tol=1e-10)
    ctx, f = B.context_from_problem(p, gmres_restart=0)
    x = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    rc, st = ctx.solve(x, f, B.SMG_VCYCLE, rtol=1e-10, maxit=100)
    assert rc == B.SMG_OK
    assert st["iterations"] == its_o
    xg = node_to_paper(host(x), p.n, p.N)
    fp = p.rhs_paper()
    assert np.linalg.norm(o.residual(xg, fp)) <= 1e-10 * np.linalg.norm(fp)
    assert_blocks(xg, x_o, p.n, p.N, 1e-12)


@pytest.mark.parametrize("n,N,seed", [(31, 8, 0), (63, 16, 1), (127, 32, 2)])
def test_gmres_solve(B, O, n, N, seed):
    p = mk(n, N, seed=seed, M=6, decay=True)
    o = O.Oracle(p)
    fp = p.rhs_paper()
    _, its_o, _ = o.gmres(fp, m=30, tol=1e-10)
    ctx, f = B.context_from_problem(p, gmres_restart=30)
    x = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    rc, st = ctx.gmres(x, f, restart=30, rtol=1e-10, maxit=100)
    assert rc == B.SMG_OK
    assert abs(st["iterations"] - its_o) <= 1
    xg = node_to_paper(host(x), n, N)
    assert np.linalg.norm(o.residual(xg, fp)) <= 1e-10 * np.linalg.norm(fp)


def test_gmres_restarts(B, O):
    """A restart length of 3 forces restarts; the explicit residual still converges."""
    p = mk(31, 8, seed=3)
    o = O.Oracle(p)
    fp = p.rhs_paper()
    _, its_o, _ = o.gmres(fp, m=3, tol=1e-10, maxit=200)
    ctx, f = B.context_from_problem(p, gmres_restart=3)
    x = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    rc, st = ctx.gmres(x, f, restart=3, rtol=1e-10, maxit=200)
    assert rc == B.SMG_OK and st["restarts"] >= 1
    assert abs(st["iterations"] - its_o) <= 2
    assert np.linalg.norm(o.residual(node_to_paper(host(x), 31, 8), fp)) <= 1e-10 * np.linalg.norm(fp)


@pytest.mark.parametrize("n,N", [(31, 8), (63, 64)])
def test_fp32_cycle_against_fp32_oracle(B, O, n, N):
    p = mk(n, N, seed=11, M=6, decay=True)
    o = O.Oracle(p)
    ctx, f = B.context_from_problem(p, gmres_restart=0, precision=B.SMG_F32)
    x_o = o.vcycle32(np.zeros(o.vlen()), p.rhs_paper(), 2)
    xd = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    ctx.vcycle(xd, f, 2)
    assert_blocks(node_to_paper(host(xd), n, N), x_o, n, N, 2e-5)


@pytest.mark.parametrize("method", [0, 1])
def test_fp32_refinement_solve(B, O, method):
    p = mk(63, 16, seed=12, M=6, decay=True)
    o = O.Oracle(p)
    fp = p.rhs_paper()
    ctx, f = B.context_from_problem(p, gmres_restart=30, precision=B.SMG_F32)
    x = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    rc, st = ctx.solve(x, f, method, rtol=1e-10, maxit=60)
    assert rc == B.SMG_OK
    xg = node_to_paper(host(x), 63, 16)
    assert np.linalg.norm(o.residual(xg, fp)) <= 1e-10 * np.linalg.norm(fp)
    x64, _, _ = o.gmres(fp, tol=1e-12)
    assert_blocks(xg, x64, 63, 16, 1e-7)
    _, its_o, inner_o, _ = o.solve_ir(fp, tol=1e-10, m=30 if method == 1 else 0)
    assert abs(st["iterations"] - its_o) <= 1


def test_single_level_is_direct_solve(B, O):
    p = mk(7, 6, seed=13)
    o = O.Oracle(p)
    ctx, f = B.context_from_problem(p, gmres_restart=0)
    x = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    rc, st = ctx.solve(x, f, B.SMG_VCYCLE, rtol=1e-12, maxit=3)
    assert rc == B.SMG_OK and st["iterations"] == 1
    S = o.assemble()
    xs = np.linalg.solve(S, p.rhs_paper())
    assert rel(node_to_paper(host(x), 7, 6), xs) <= 1e-11


def test_error_paths(B):
    p = mk(15, 2, seed=14)
    kxn, kyn = p.faces_node()
    kx = dev(kxn); ky = dev(kyn)
    bad = kx.clone(); bad[3] = -1.0
    with pytest.raises(B.SmgError) as ei:
        B.Context(15, 2, bad, ky, p.c, p.d, p.e, p.g, gmres_restart=0)
    assert ei.value.code == -2
    with pytest.raises(B.SmgError):
        B.Context(15, 2, kx, ky, p.c, p.d, p.e, -1.0, gmres_restart=0)
    ctx = B.Context(15, 2, kx, ky, p.c, p.d, p.e, p.g, gmres_restart=0)
    f = dev(p.rhs_node())
    f[5] = float("nan")
    x = torch.zeros_like(f)
    with pytest.raises(B.SmgError) as ei:
        ctx.solve(x, f, B.SMG_VCYCLE, rtol=1e-10, maxit=5)
    assert ei.value.code == -4
    f = dev(p.rhs_node())
    rc, st = ctx.solve(torch.zeros_like(f), f, B.SMG_VCYCLE, rtol=1e-10, maxit=1)
    assert rc == B.SMG_NOT_CONVERGED and st["iterations"] == 1
    last = ctx.nlev - 1     # the coarsest level has no coarser one to restrict to
    with pytest.raises(B.SmgError) as ei:
        ctx.residual_restrict(last, x, f, x)
    assert ei.value.code == -1


def test_medium_size_cycle_against_oracle(B, O):
    """255x255, N = 64: one and two V-cycles from zero match the oracle in every
    block (Y, U, P), in the launch configuration of the solver."""
    p = inputs.medium_fp64()
    o = O.Oracle(p)
    ctx, f = B.context_from_problem(p, gmres_restart=30)
    x_o = np.zeros(o.vlen())
    xd = torch.zeros(o.vlen(), dtype=torch.float64, device="cuda")
    for k in range(2):
        x_o = o.vcycle(x_o, p.rhs_paper(), 1)
        ctx.vcycle(xd, f, 1)
        assert_blocks(node_to_paper(host(xd), p.n, p.N), x_o, p.n, p.N, 1e-12, k)


@pytest.mark.parametrize("n,N", [(63, 16), (31, 100), (15, 256)])
def test_fp32_halfsweeps_against_fp32_oracle(B, O, n, N):
    """The FP32 smoother (smg_smooth32) against the oracle's half-sweep in FP32
    arithmetic from the same FP32-rounded iterate: agreement to FP32 rounding."""
    p = mk(n, N, seed=3 * n + N)
    o = O.Oracle(p, coarsest_n=7)
    ctx, _ = B.context_from_problem(p, gmres_restart=0, precision=B.SMG_F32)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(o.vlen()).astype(np.float32).astype(np.float64)
    fp = p.rhs_paper().astype(np.float32).astype(np.float64)
    xd = torch.from_numpy(paper_to_node(x, n, N).astype(np.float32)).cuda()
    fd = torch.from_numpy(paper_to_node(fp, n, N).astype(np.float32)).cuda()
    for colour in (0, 1, 0, 1):
        x = o.halfsweep32(x, fp, colour)
        ctx.smooth32(0, colour, xd, fd)
        got = node_to_paper(host(xd).astype(np.float64), n, N)
        assert rel(got, x) <= 2e-6, colour
    with pytest.raises(B.SmgError):
        c64, _ = B.context_from_problem(p, gmres_restart=0)
        c64.smooth32(0, 0, xd, fd)
