"""The one-launch red+black sweep (k_sweep_fused) against the two half-sweeps it
replaces and against the oracle: single sweeps on every level that takes it,
with segment boundaries forced by short segments, in FP64 and FP32, and whole
V-cycles with and without it."""
import numpy as np
import pytest

from paper_2302_13680_amd import inputs
from paper_2302_13680_amd.inputs import node_to_paper, paper_to_node
from parity_util import assert_blocks, block_rel

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


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("n,N,rows", [(127, 64, 200), (127, 100, 5), (255, 64, 16), (127, 256, 64), (255, 33, 7)])
def test_sweep_equals_two_halfsweeps_and_oracle(B, O, n, N, rows):
    p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=n + N)
    o = O.Oracle(p)
    ctx, _ = B.context_from_problem(p, gmres_restart=0, sweep_rows=rows)
    rng = np.random.default_rng(N)
    x = rng.standard_normal(o.vlen())
    f = rng.standard_normal(o.vlen())
    xd, fd = dev(paper_to_node(x, n, N)), dev(paper_to_node(f, n, N))
    out = torch.empty_like(xd)
    assert ctx.sweep(0, xd, out, fd)                      # one launch on this level
    ref = xd.clone()
    ctx.smooth(0, 0, ref, fd)
    ctx.smooth(0, 1, ref, fd)
    got = node_to_paper(host(out), n, N)
    assert_blocks(got, node_to_paper(host(ref), n, N), n, N, 1e-15, "two half-sweeps")
    xo = o.halfsweep(o.halfsweep(x, f, 0), f, 1)
    assert_blocks(got, xo, n, N, 1e-13, "oracle")


@pytest.mark.parametrize("n,N", [(63, 256), (63, 200), (31, 193), (127, 100), (15, 130)])
def test_column_walk_residual_restrict_against_oracle(B, O, n, N):
    """Where the sweeps run in one launch the V-cycle's residual + restriction
    walks columns (k_rr_walk): every level against the oracle's residual then
    full weighting, per block, with random x and f (even, odd and ragged N;
    the short levels give one coarse row per segment)."""
    p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=3 * n + N)
    o = O.Oracle(p)
    ctx, _ = B.context_from_problem(p, gmres_restart=0, sweep_rows=4)
    rng = np.random.default_rng(n + N)
    for l in range(o.nlev - 1):
        nl, nc = o.levels_n[l], o.levels_n[l + 1]
        x = rng.standard_normal((2 * N + 1) * nl * nl)
        f = rng.standard_normal(x.size)
        cd = torch.empty((2 * N + 1) * nc * nc, dtype=torch.float64, device="cuda")
        ctx.residual_restrict(l, dev(paper_to_node(x, nl, N)), dev(paper_to_node(f, nl, N)), cd)
        ref = O.restrict(nl, N, o.residual(x, f, l))
        assert_blocks(node_to_paper(host(cd), nc, N), ref, nc, N, 1e-14, f"level {l}")


@pytest.mark.parametrize("n,N", [(63, 256), (63, 200), (31, 193), (127, 100), (15, 130), (63, 64), (31, 65),
                                 (15, 255), (31, 129)])
def test_restriction_after_sweep_from_the_black_change(B, O, n, N):
    """Where the column walk applies, the restriction after a sweep x0 -> x1
    (k_rr_gs_walk: from the blacks' change, f not read) against the oracle's
    R (f - S x1) on every level, x1 the oracle's own sweep of random x0: Y and P
    blocks on their own scale; the U block exactly zero on the GPU and at the
    rounding level in the oracle.  N = 64: one sample per lane; 100, 200, 256:
    two per access; 65, 129, 130, 193, 255: one at a time with a ragged tail."""
    p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=5 * n + N)
    o = O.Oracle(p)
    ctx, _ = B.context_from_problem(p, gmres_restart=0, sweep_rows=4)
    rng = np.random.default_rng(n * N)
    for l in range(o.nlev - 1):
        nl, nc = o.levels_n[l], o.levels_n[l + 1]
        x0 = rng.standard_normal(o.vlen(l))
        f = rng.standard_normal(o.vlen(l))
        x1 = o.halfsweep(o.halfsweep(x0, f, 0, l), f, 1, l)
        cd = torch.full((o.vlen(l + 1),), np.nan, dtype=torch.float64, device="cuda")
        walk = ctx.residual_restrict_after_sweep(l, dev(paper_to_node(x0, nl, N)), dev(paper_to_node(x1, nl, N)),
                                                 dev(paper_to_node(f, nl, N)), cd)
        assert walk, l
        got = node_to_paper(host(cd), nc, N)
        ref = O.restrict(nl, N, o.residual(x1, f, l))
        e = block_rel(got, ref, nc, N)
        print("level", l, e, flush=True)
        assert e["y"] <= 1e-12 and e["p"] <= 1e-12, (l, e)
        ncn = nc * nc
        assert np.all(got[N * ncn:(N + 1) * ncn] == 0.0)
        assert np.linalg.norm(ref[N * ncn:(N + 1) * ncn]) <= 1e-12 * np.linalg.norm(ref)


def test_restriction_after_sweep_without_the_walk_reads_f(B, O):
    """63 x 63, N = 64 without a forced segment length: no column walk, so the
    entry point forms R (f - S x1) from f (the plain fused pass)."""
    n, N = 63, 64
    p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=9)
    o = O.Oracle(p)
    ctx, _ = B.context_from_problem(p, gmres_restart=0)
    rng = np.random.default_rng(9)
    x0 = rng.standard_normal(o.vlen())
    f = rng.standard_normal(o.vlen())
    x1 = o.halfsweep(o.halfsweep(x0, f, 0), f, 1)
    nc = o.levels_n[1]
    cd = torch.empty(o.vlen(1), dtype=torch.float64, device="cuda")
    assert not ctx.residual_restrict_after_sweep(0, dev(paper_to_node(x0, n, N)), dev(paper_to_node(x1, n, N)),
                                                 dev(paper_to_node(f, n, N)), cd)
    got, ref = node_to_paper(host(cd), nc, N), o.residual_restrict(x1, f)
    e = block_rel(got, ref, nc, N)
    assert e["y"] <= 1e-13 and e["p"] <= 1e-13, e
    # after a sweep the U rows vanish: both sides leave only rounding there
    ncn = nc * nc
    for v in (got, ref):
        assert np.linalg.norm(v[N * ncn:(N + 1) * ncn]) <= 1e-12 * np.linalg.norm(ref)
    xa = dev(paper_to_node(x0, n, N))
    with pytest.raises(B.SmgError):                       # xold and xnew the same vector
        ctx.residual_restrict_after_sweep(0, xa, xa, dev(paper_to_node(f, n, N)), cd)


@pytest.mark.parametrize("n,N", [(63, 256), (63, 200), (31, 193), (127, 100), (63, 64), (15, 130), (31, 65),
                                 (15, 255), (31, 129)])
def test_column_walk_residual_and_apply_equal_the_per_node_form(B, O, n, N):
    """On one-launch levels the finest residual and operator application run in
    column walks (k_residual_walk): with the per-node arithmetic, so the vectors
    equal those of the per-node kernel bit for bit (a context without forced
    segments at these sizes), the block norms to the summation order, and the
    oracle's residual per block.  Even, odd and ragged N."""
    p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=7 * n + N)
    o = O.Oracle(p)
    cw, _ = B.context_from_problem(p, gmres_restart=0, sweep_rows=4)
    cn, _ = B.context_from_problem(p, gmres_restart=0)
    rng = np.random.default_rng(3 * n + N)
    x = rng.standard_normal(o.vlen())
    f = rng.standard_normal(o.vlen())
    xd, fd = dev(paper_to_node(x, n, N)), dev(paper_to_node(f, n, N))
    a1, a2 = torch.empty_like(xd), torch.empty_like(xd)
    cw.apply(xd, a1)
    cn.apply(xd, a2)
    assert torch.equal(a1, a2)
    r1, r2 = torch.empty_like(xd), torch.empty_like(xd)
    h1 = cw.residual(xd, fd, r1, norms=True)
    h2 = cn.residual(xd, fd, r2, norms=True)
    assert torch.equal(r1, r2)
    np.testing.assert_allclose(h1, h2, rtol=1e-13)
    assert_blocks(node_to_paper(host(r1), n, N), o.residual(x, f), n, N, 1e-14, "oracle residual")
    assert_blocks(node_to_paper(host(a1), n, N), o.apply(x), n, N, 1e-14, "oracle apply")


@pytest.mark.parametrize("N", [200, 193])
def test_fp32_fgmres_with_column_walks(B, O, N):
    """FGMRES(30) around FP32 cycles where the operator application on FP32
    preconditioned vectors runs in column walks (forced by a segment length):
    the solution meets 1e-10 in the oracle's FP64 residual, with the oracle's
    refinement count within one."""
    p = inputs.make_problem(127, N, 1e-4, M=6, sigma=0.5, decay=True, seed=6)
    o = O.Oracle(p)
    ctx, f = B.context_from_problem(p, gmres_restart=30, precision=B.SMG_F32, sweep_rows=8)
    x = torch.zeros(p.dof, dtype=torch.float64, device="cuda")
    rc, st = ctx.solve(x, f, B.SMG_GMRES, rtol=1e-10, maxit=60)
    assert rc == B.SMG_OK, st
    fp = p.rhs_paper()
    r = o.residual(node_to_paper(host(x), p.n, p.N), fp)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(fp)
    _, its, _, _ = o.solve_ir(fp, tol=1e-10, m=30)
    assert abs(st["iterations"] - its) <= 1, (st["iterations"], its)


@pytest.mark.parametrize("case", ["local control", "theta 1/2"])
def test_restriction_after_sweep_falls_back_where_the_identity_is_not_used(B, O, case):
    """With node factors (control on a subregion) or theta != 1 the entry point
    forms R (f - S xnew) from f (the black-change form needs plain Gauss-Seidel
    rows without factors): it reports so, even with forced segments, and matches
    the oracle's fused residual + restriction for any xnew."""
    n, N = 63, 200
    if case == "local control":
        p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=41,
                                control_region=(0.25, 0.75, 0.25, 0.75))
        ctx, _ = B.context_from_problem(p, gmres_restart=0, sweep_rows=8)
    else:
        p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=42)
        ctx, _ = B.context_from_problem(p, gmres_restart=0, sweep_rows=8, theta=0.5)
    o = O.Oracle(p)
    rng = np.random.default_rng(43)
    x0 = rng.standard_normal(o.vlen())
    x1 = rng.standard_normal(o.vlen())
    f = rng.standard_normal(o.vlen())
    nc = o.levels_n[1]
    cd = torch.empty(o.vlen(1), dtype=torch.float64, device="cuda")
    assert not ctx.residual_restrict_after_sweep(0, dev(paper_to_node(x0, n, N)), dev(paper_to_node(x1, n, N)),
                                                 dev(paper_to_node(f, n, N)), cd)
    assert_blocks(node_to_paper(host(cd), nc, N), o.residual_restrict(x1, f), nc, N, 1e-13, case)


def test_sweep_refuses_aliasing_and_reports_the_fallback(B):
    p = inputs.make_problem(63, 64, 1e-4, M=6, sigma=0.5, decay=True, seed=3)
    ctx, f = B.context_from_problem(p, gmres_restart=0)
    x = torch.zeros(p.dof, dtype=torch.float64, device="cuda")
    with pytest.raises(B.SmgError):
        ctx.sweep(0, x, x, f)
    out = torch.empty_like(x)
    assert not ctx.sweep(0, x, out, f)                    # 63 x 63: two half-sweeps


@pytest.mark.parametrize("n,N", [(127, 128), (255, 256)])
def test_fp32_sweep_equals_two_halfsweeps(B, O, n, N):
    p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=7)
    o = O.Oracle(p)
    ctx, _ = B.context_from_problem(p, gmres_restart=0, precision=B.SMG_F32, sweep_rows=32)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(o.vlen())
    f = rng.standard_normal(o.vlen())
    xd, fd = dev(paper_to_node(x, n, N), torch.float32), dev(paper_to_node(f, n, N), torch.float32)
    out = torch.empty_like(xd)
    assert ctx.sweep32(0, xd, out, fd)
    ref = xd.clone()
    ctx.smooth32(0, 0, ref, fd)
    ctx.smooth32(0, 1, ref, fd)
    assert_blocks(node_to_paper(host(out), n, N), node_to_paper(host(ref), n, N), n, N, 1e-7, "two half-sweeps")
    xo = o.halfsweep32(o.halfsweep32(x, f, 0), f, 1)
    assert_blocks(node_to_paper(host(out), n, N), xo, n, N, 2e-6, "oracle")


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n,N", [(255, 64), (127, 200), (127, 193)])
def test_vcycles_with_and_without_one_launch_sweeps(B, O, precision, n, N):
    """32-row segments: every level sweeps in one launch (zero start on the
    coarse levels, the coarse correction added at the black nodes ahead of
    post-smoothing, the residual restricted in column walks); iterates equal
    those of the half-sweep cycle and the oracle's.  N = 64: one sample per
    lane; 200: four per lane in pairs (16-byte FP64 accesses) with a ragged
    tail; 193: four per lane one at a time."""
    p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=21)
    o = O.Oracle(p)
    fp = p.rhs_paper()
    c1, f = B.context_from_problem(p, gmres_restart=0, precision=precision, sweep_rows=32)
    c2, _ = B.context_from_problem(p, gmres_restart=0, precision=precision, flags=B.SMG_FLAG_HALFSWEEPS)
    x1 = torch.zeros(p.dof, dtype=torch.float64, device="cuda")
    x2 = torch.zeros_like(x1)
    xo = np.zeros(o.vlen())
    cyc = o.vcycle if precision == 0 else o.vcycle32
    # FP32: two single-precision evaluations of the same cycle differ by rounding
    # (unit roundoff 6e-8) amplified by the cancellation in p_j = (b_P - c_j y_j) / a_j,
    # where b_P and c_j y_j are ~1e3 times p_j: ~1e-5 relative in the P block
    tol_pair, tol_or = (1e-13, 1e-12) if precision == 0 else (1e-4, 1e-4)
    for k in range(2):
        c1.vcycle(x1, f, 1)
        c2.vcycle(x2, f, 1)
        xo = cyc(xo, fp, 1)
        g1 = node_to_paper(host(x1), p.n, p.N)
        e1 = assert_blocks(g1, node_to_paper(host(x2), p.n, p.N), p.n, p.N, tol_pair, k)
        e2 = assert_blocks(g1, xo, p.n, p.N, tol_or, k)
        print("cycle", k, "one-launch vs half-sweeps", e1, "vs oracle", e2, flush=True)


@pytest.mark.parametrize("pre,post", [(1, 1), (3, 3), (1, 2), (3, 1), (2, 3)])
def test_vcycles_with_odd_smoothing_counts(B, O, pre, post):
    """Odd numbers of sweeps on one-launch levels: the first sweep then runs as two
    half-sweeps in place and the rest in one-launch pairs (blacks-only stores but
    for the cycle's last sweep, the restriction from the blacks' change only after
    two or more pre-smoothing sweeps); iterates against the half-sweep cycle and
    the oracle with the same counts, every cycle, per block."""
    n, N = 127, 200
    p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=31)
    o = O.Oracle(p, pre=pre, post=post)
    fp = p.rhs_paper()
    c1, f = B.context_from_problem(p, gmres_restart=0, pre=pre, post=post, sweep_rows=16)
    c2, _ = B.context_from_problem(p, gmres_restart=0, pre=pre, post=post, flags=B.SMG_FLAG_HALFSWEEPS)
    x1 = torch.zeros(p.dof, dtype=torch.float64, device="cuda")
    x2 = torch.zeros_like(x1)
    xo = np.zeros(o.vlen())
    for k in range(2):
        c1.vcycle(x1, f, 1)
        c2.vcycle(x2, f, 1)
        xo = o.vcycle(xo, fp, 1)
        g1 = node_to_paper(host(x1), n, N)
        assert_blocks(g1, node_to_paper(host(x2), n, N), n, N, 1e-13, ("half-sweeps", k))
        assert_blocks(g1, xo, n, N, 1e-12, ("oracle", k))


@pytest.mark.parametrize("N", [256, 128])
def test_large_level_takes_the_one_launch_sweep_by_default(B, N):
    """511x511, N = 256 or 128 (levels that stream from HBM; four or two samples
    per lane): the default context sweeps in one launch, SMG_FLAG_HALFSWEEPS does
    not, and both give the same sweep."""
    p = inputs.large_mixed() if N == 256 else inputs.make_problem(511, N, 1e-4, M=6, sigma=1.0, decay=True, seed=2)
    ctx, f = B.context_from_problem(p, gmres_restart=0)
    xin = torch.rand(p.dof, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    a = torch.empty_like(xin)
    assert ctx.sweep(0, xin, a, f)
    ctx.close()
    c2, _ = B.context_from_problem(p, gmres_restart=0, flags=B.SMG_FLAG_HALFSWEEPS)
    b = torch.empty_like(xin)
    assert not c2.sweep(0, xin, b, f)
    rel = (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item()
    assert rel <= 1e-15, rel


@pytest.mark.parametrize("N", [200, 193])
def test_fp32_refinement_with_column_walks(B, O, N):
    """FP32 cycles in FP64 refinement where the refinement residual runs in column
    walks (k_residual_add_walk, forced here by a segment length): the solution meets
    1e-10 in the oracle's FP64 residual, in total and per block row, with the
    oracle's refinement count within one."""
    p = inputs.make_problem(127, N, 1e-4, M=6, sigma=0.5, decay=True, seed=5)
    o = O.Oracle(p)
    ctx, f = B.context_from_problem(p, gmres_restart=0, precision=B.SMG_F32, sweep_rows=8)
    x = torch.zeros(p.dof, dtype=torch.float64, device="cuda")
    rc, st = ctx.solve(x, f, B.SMG_VCYCLE, rtol=1e-10, maxit=60)
    assert rc == B.SMG_OK, st
    fp = p.rhs_paper()
    xg = node_to_paper(host(x), p.n, p.N)
    r = o.residual(xg, fp)
    nf = np.linalg.norm(fp)
    nn = p.n * p.n
    assert np.linalg.norm(r) <= 1e-10 * nf
    for blk in (r[:N * nn], r[N * nn:(N + 1) * nn], r[(N + 1) * nn:]):
        assert np.linalg.norm(blk) <= 1e-10 * nf
    _, its, _, _ = o.solve_ir(fp, tol=1e-10, m=0)
    assert abs(st["iterations"] - its) <= 1, (st["iterations"], its)
