"""Benchmark of the collective multigrid solver on one MI355X.

One step = one full solve of the 511x511, N = 256 linear-quadratic OCPUU
(FP64, six KL modes of amplitude 1.0/m, nu = 1e-4; 1.34e8 unknowns) from a
zero initial guess to a relative residual of 1e-8 with GMRES(30) preconditioned
by one V(2,2) cycle, inputs resident in HBM.

Output: one JSON line per further section (255x255 figures, batched and
learned forms, the paper's table settings), then the headline record as the
LAST line:

value  = whole-job DoF-sweeps/s: (2N+1) n^2 unknowns x fine-level smoothing
         sweeps performed in the solve (4 per V-cycle) / solve wall time.
roofline: the dominant kernel (the collective Gauss-Seidel half-sweep on the
         finest level) timed with HIP events on the library's stream, priced at
         half of a red+black sweep's algorithmic bytes (8 words per
         node-sample, 2 per node) against the 8 TB/s HBM peak.
cpu_baseline: the FP64 CPU oracle on the same instance (V(2,2) cycles from
         zero, about 10 s of CPU work) on the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time to rel. residual 1e-8 & DoF-sweeps/s; % HBM roofline; vs plain FP64 V-cycle")
HBM_PEAK_GBS = 8000.0


def kernel_source_hash() -> str:
    """Hash of the sources the finest-level sweep kernels are built from."""
    h = hashlib.sha256()
    for f in ("common.h", "smoother.h", "sweep.h"):
        with open(os.path.join(ROOT, "paper_2302_13680_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def halfsweep_bytes(n: int, N: int, word: int) -> float:
    """Algorithmic bytes of one half-sweep launch (red colour): the 4 faces of
    every updated node, y and p of every node of the other colour, the three
    right-hand-side rows of the updated nodes, and y, p, u written back."""
    nact = ((n - 1) // 2) * n + (n + 1) // 2
    nin = n * n - nact
    words = N * (4 * nact + 2 * nin + 2 * nact + 2 * nact) + 2 * nact
    return float(words * word)


def load_traffic(kind: str):
    path = os.path.join(ROOT, "profiles", f"traffic_{kind}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_hash") != kernel_source_hash():
        return None     # the kernel changed since the counters were taken
    return t.get("bytes_per_launch")


def time_halfsweep(ctx, x, f, stream, launches, fp32=False):
    """Average duration (us) of `launches` finest-level half-sweeps, HIP events on
    the library's stream (fp32: the FP32 smoother on float32 vectors)."""
    import torch
    smooth = ctx.smooth32 if fp32 else ctx.smooth
    for _ in range(5):
        smooth(0, 0, x, f)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(launches):
        smooth(0, i & 1, x, f)
    e1.record(stream)
    e1.synchronize()
    return 1e3 * e0.elapsed_time(e1) / launches


def halfsweep_counter_run(ctx, x, f, n, N):
    """20 finest-level sweeps (one launch each where the level takes the
    one-launch sweep, else 40 half-sweeps), finest-level residuals and
    residual + restrictions (from f, then from the last sweep's change of the
    black nodes), 2 V-cycles, then five 1 GiB device copies (the calibration of
    the traffic counters)."""
    import torch
    xb = torch.empty_like(x)
    one = ctx.sweep(0, x, xb, f)
    for i in range(19):
        if one:
            ctx.sweep(0, xb, x, f) if i % 2 == 0 else ctx.sweep(0, x, xb, f)
        else:
            ctx.smooth(0, 0, x, f)
            ctx.smooth(0, 1, x, f)
    # the other finest-level passes of a cycle: 5 operator residuals (r written,
    # norms), 5 + 5 fused residual + restrictions, then 2 V-cycles (zero-start and
    # plain sweeps, the black-node prolongation, every coarser level)
    r = torch.empty_like(x)
    coarse = torch.empty(ctx.vlen(1), dtype=torch.float64, device=x.device)
    for _ in range(5):
        ctx.residual(x, f, r, norms=True)
    for _ in range(5):
        ctx.residual_restrict(0, x, f, coarse)
    if one:   # x is the last sweep of xb: the restriction from the blacks' change
        for _ in range(5):
            ctx.residual_restrict_after_sweep(0, xb, x, f, coarse)
    ctx.vcycle(x, f, 2)
    a = torch.ones(1 << 27, dtype=torch.float64, device=x.device)   # 1 GiB
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"counters": "done", "n": n, "N": N, "one_launch_sweeps": one,
                      "sweep_algorithmic_bytes": sweep_bytes(n, N, 8),
                      "copy_bytes_each_way": a.numel() * 8, "copy_launches": 5}), flush=True)


def timed_solve(ctx, x, f, method, rtol, maxit=200):
    import torch
    from paper_2302_13680_amd import binding
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = ctx.solve(x, f, method, rtol=rtol, maxit=maxit, history=0)
    torch.cuda.synchronize()
    if rc != binding.SMG_OK:
        raise RuntimeError(f"solve did not converge: {st}")
    return 1e3 * (time.perf_counter() - t0), st


def large_mixed_section(dev):
    """511x511, N=256, six modes of amplitude 1.0/m: FP32 V-cycle inside FP64
    refinement against the plain FP64 V-cycle on the same GPU."""
    import torch
    from paper_2302_13680_amd import binding, inputs
    prob = inputs.large_mixed()
    n, N, dof = prob.n, prob.N, prob.dof
    kxn, kyn = prob.faces_node()
    kx = torch.from_numpy(kxn).to(dev)
    ky = torch.from_numpy(kyn).to(dev)
    f = torch.from_numpy(prob.rhs_node()).to(dev)
    del kxn, kyn
    c64 = binding.Context(n, N, kx, ky, prob.c, prob.d, prob.e, prob.g, gmres_restart=0)
    c32 = binding.Context(n, N, kx, ky, prob.c, prob.d, prob.e, prob.g, gmres_restart=30,
                          precision=binding.SMG_F32)
    x = torch.zeros(dof, dtype=torch.float64, device=dev)
    out = {"workload": "LQ-OCPUU 511x511 interior grid, N=256 samples, 6 KL modes a_m=1.0/m, nu=1e-4",
           "dof": dof}
    timed_solve(c64, x, f, binding.SMG_VCYCLE, 1e-8)          # warm-up (graph capture)
    t64, s64 = timed_solve(c64, x, f, binding.SMG_VCYCLE, 1e-8)
    out["fp64_vcycle_time_to_1e-8_ms"] = round(t64, 2)
    out["fp64_vcycle_cycles"] = s64["iterations"]
    for name, method in (("fp32_refinement_vcycle", binding.SMG_VCYCLE), ("fp32_refinement_fgmres30", binding.SMG_GMRES)):
        timed_solve(c32, x, f, method, 1e-8)
        t, st = timed_solve(c32, x, f, method, 1e-8)
        out[name + "_time_to_1e-8_ms"] = round(t, 2)
        out[name + "_outer_steps"] = st["iterations"]
        out[name + "_fp32_cycles"] = st["inner_iterations"]
        out[name + "_speedup_vs_fp64_vcycle"] = round(t64 / t, 3)
    # errors at 1e-10: FP32 refinement against the FP64 V-cycle solution
    t64b, _ = timed_solve(c64, x, f, binding.SMG_VCYCLE, 1e-10)
    x64 = x.clone()
    t32b, st32b = timed_solve(c32, x, f, binding.SMG_VCYCLE, 1e-10)
    out["fp64_vcycle_time_to_1e-10_ms"] = round(t64b, 2)
    out["fp32_refinement_vcycle_time_to_1e-10_ms"] = round(t32b, 2)
    nn = n * n
    blocks = {"y": slice(0, N * nn), "u": slice(N * nn, (N + 1) * nn), "p": slice((N + 1) * nn, None)}
    out["fp32_refinement_rel_diff_vs_fp64_at_1e-10"] = {
        k: float((torch.linalg.norm(x[sl] - x64[sl]) / torch.linalg.norm(x64[sl])).item()) for k, sl in blocks.items()}
    # finest-level sweeps in both precisions: the one-launch sweep and the two
    # half-sweeps, priced at a sweep's algorithmic bytes (8 words per node-sample)
    for name, ctx, dt, w in (("fp64", c64, torch.float64, 8), ("fp32", c32, torch.float32, 4)):
        xa = torch.zeros(dof, dtype=dt, device=dev)
        xb = torch.empty_like(xa)
        fx = f if dt == torch.float64 else f.float()
        fp32 = dt == torch.float32
        one = (ctx.sweep32 if fp32 else ctx.sweep)(0, xa, xb, fx)
        rec = {}
        if one:
            us1 = time_sweep(ctx, xa, xb, fx, ctx.stream, 40, fp32=fp32)
            rec["one_launch_us"] = round(us1, 2)
            rec["one_launch_frac_of_8TBs"] = round(sweep_bytes(n, N, w) / (us1 * 1e-6) / 8e12, 4)
        us2 = 2 * time_halfsweep(ctx, xa, fx, ctx.stream, 40, fp32=fp32)
        rec["two_halfsweeps_us"] = round(us2, 2)
        rec["two_halfsweeps_frac_of_8TBs"] = round(sweep_bytes(n, N, w) / (us2 * 1e-6) / 8e12, 4)
        out["sweep_" + name] = rec
        del xa, xb
    del x64
    return out, c32, f, x


def large_ssn_section(dev):
    """Algorithm 2 at 511x511, N=256 (the paper's target, nu 1e-4, beta 1e-2,
    |u| <= 50): stationary V-cycle inner solves in FP64 against FP64 refinement
    around FP32 cycles.  The inner tolerance is 1e-10: at this size (1.3e8
    unknowns) the Newton systems' FP64 residual floor is ~1.2e-11 relative,
    above the 1e-11 used at the paper's sizes."""
    import torch
    from paper_2302_13680_amd import binding, inputs
    p = inputs.make_problem(511, 256, 1e-4, M=6, sigma=1.0, decay=True, seed=2, yd=inputs.paper_target(511), f=0.0)
    out = {"problem": "511x511, N=256, nu=1e-4, beta=1e-2, -50 <= u <= 50, y_d = exp(y^2) sin 2pi x sin 2pi y, f=0",
           "inner": "stationary V(2,2) to 1e-10"}
    h2 = (1.0 / 512) ** 2
    prm = binding.ssn_params(1e-4, 1e-2, -50.0, 50.0, h2, inner_rtol=1e-10, inner_method=binding.SMG_VCYCLE)
    t64 = None
    for name, prec in (("fp64", binding.SMG_F64), ("fp32_refinement", binding.SMG_F32)):
        ctx, f = binding.context_from_problem(p, device=dev, gmres_restart=0, ssn=True, precision=prec)
        x = torch.zeros(p.dof, dtype=torch.float64, device=dev)
        ssn_run(ctx, x, f, prm)                                    # warm-up (graph capture)
        t, rc, st = ssn_run(ctx, x, f, prm)
        out[name] = {"time_ms": round(t, 1), "converged": rc == binding.SMG_OK, "newton_iterations": st["iterations"],
                     "inner_iterations": st["inner"], "initial_solve_iterations": st["init_iterations"],
                     "phi_final": st["phi_final"]}
        if t64 is None:
            t64 = t
        else:
            out[name]["speedup_vs_fp64"] = round(t64 / t, 3)
        ctx.close()
        del ctx, f, x
        torch.cuda.empty_cache()
    return out


def batch_section(dev, cache_path):
    """64 uneven instances (n in {63,127,255}, N in {16,32,64,128}, nu log-uniform
    in [1e-6, 1e-2]) solved to 1e-8 by the batched FP32-refined solver with
    autotuned lane widths, against sequential plain FP64 V-cycle solves."""
    import torch
    from paper_2302_13680_amd import autotune, binding, inputs
    specs = inputs.batch_instances()
    c32s, c64s, xs, fs = [], [], [], []
    for sp in specs:
        p = inputs.make_problem(sp["n"], sp["N"], sp["nu"], M=6, sigma=0.5, decay=True, seed=sp["seed"])
        kxn, kyn = p.faces_node()
        kx = torch.from_numpy(kxn).to(dev)
        ky = torch.from_numpy(kyn).to(dev)
        f = torch.from_numpy(p.rhs_node()).to(dev)
        c32s.append(binding.Context(p.n, p.N, kx, ky, p.c, p.d, p.e, p.g, gmres_restart=0,
                                    precision=binding.SMG_F32))
        c64s.append(binding.Context(p.n, p.N, kx, ky, p.c, p.d, p.e, p.g, gmres_restart=0))
        xs.append(torch.zeros(p.dof, dtype=torch.float64, device=dev))
        fs.append(f)
    t0 = time.perf_counter()
    lanes, _ = autotune.tune(c32s, cache_path)
    t_tune = time.perf_counter() - t0
    bt = binding.Batch(c32s, xs, fs, lanes=lanes)
    for x in xs:
        x.zero_()
    bt.solve(rtol=1e-8, maxit=60)                        # warm-up (graph capture)
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, stats, wall = bt.solve(rtol=1e-8, maxit=60)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    # sequential plain FP64 V-cycle solves of the same instances on the same GPU
    for c, x, f in zip(c64s, xs, fs):
        timed_solve(c, x, f, binding.SMG_VCYCLE, 1e-8)   # warm-up (graph capture)
    t0 = time.perf_counter()
    seq = []
    for c, x, f in zip(c64s, xs, fs):
        t, st = timed_solve(c, x, f, binding.SMG_VCYCLE, 1e-8)
        seq.append(t)
    t_seq = time.perf_counter() - t0
    return {
        "workload": "64 LQ-OCPUU instances, n in {63,127,255}, N in {16,32,64,128}, nu log-uniform [1e-6,1e-2], "
                    "6 KL modes a_m=0.5/m, FP32 V(2,2) in FP64 refinement to 1e-8",
        "converged": rc == 0, "instances": len(specs), "wall_ms": round(1e3 * t_batch, 2),
        "aggregate_solves_per_s": round(len(specs) / t_batch, 2),
        "sequential_fp64_vcycle_ms": round(1e3 * t_seq, 2),
        "speedup_vs_sequential_fp64_vcycle": round(t_seq / t_batch, 3),
        "autotune_s": round(t_tune, 2), "lanes": lanes,
        "per_instance": [{"n": sp["n"], "N": sp["N"], "nu": sp["nu"], "cycles": st["iterations"],
                          "time_to_1e-8_ms": round(st["time_ms"], 3), "fp64_vcycle_ms": round(t, 3)}
                         for sp, st, t in zip(specs, stats, seq)],
    }


def learned_section(dev, n_train=2000, n_test=200, epochs=20):
    """Warm start on 127x127, N=128 (nu log-uniform in [1e-5, 1e-3], y_d random
    sums of three sine products): 2000 multigrid solves as training data, the
    network trained on the GPU by the library's kernels, 200 held-out seeds,
    checked after one V-cycle against the zero start's first-cycle residual."""
    import numpy as np
    import torch
    from paper_2302_13680_amd import binding, learn
    n, N = 127, 128
    H = learn.grid_for(n)
    t0 = time.perf_counter()
    first = []
    feats, raw = learn.make_dataset(list(range(10000, 10000 + n_train)), n=n, N=N, device=dev, first_cycle=first)
    t_data = time.perf_counter() - t0
    rho0 = float(np.median(first))
    norm = learn.standardization(raw, n)
    tg = learn.standardize(raw, norm, n)
    del raw
    net = binding.Net(16, H, device=dev)
    net.set_params(torch.tensor(learn.param_init(0), device=dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = learn.train(net, feats, tg, n, epochs=epochs, lr=2e-3, seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del feats, tg
    recs = learn.evaluate(net, list(range(20000, 20000 + n_test)), norm, n=n, N=N, device=dev, rho0=rho0)
    summ = learn.summarize(recs)
    summ.update({"workload": "127x127, N=128, nu log-uniform [1e-5,1e-3], y_d random sums of 3 sine "
                             "products; FP64 V(2,2) to 1e-8",
                 "params": net.np, "train_instances": n_train, "test_instances": n_test,
                 "epochs": epochs, "dataset_s": round(t_data, 2), "train_s": round(t_train, 2),
                 "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1]})
    return summ


def ssn_run(ctx, x, f, prm, u0=None):
    """One timed smg_ssn_solve from u0 (zero) with zero state and adjoint guesses."""
    import numpy as np
    import torch
    from paper_2302_13680_amd import binding, inputs
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = ctx.ssn_solve(x, f, prm)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0), rc, st


def ssn_section(dev, n, N, args):
    import numpy as np
    import torch
    from paper_2302_13680_amd import binding, inputs
    p = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=1, yd=inputs.paper_target(n), f=0.0)
    ctx, f = binding.context_from_problem(p, device=dev, gmres_restart=30, ssn=True)
    x = torch.zeros(p.dof, dtype=torch.float64, device=dev)
    h2 = (1.0 / (n + 1)) ** 2
    out = {"problem": f"{n}x{n}, N={N}, nu=1e-4, beta=1e-2, -50 <= u <= 50, y_d = exp(y^2) sin 2pi x sin 2pi y, f=0",
           "tol_phi": 1e-9, "inner_rtol": 1e-11}
    for name, method in (("gmres30", binding.SMG_GMRES), ("vcycle", binding.SMG_VCYCLE)):
        prm = binding.ssn_params(1e-4, 1e-2, -50.0, 50.0, h2, inner_method=method)
        ssn_run(ctx, x, f, prm)                                    # warm-up (graph capture)
        t, rc, st = ssn_run(ctx, x, f, prm)
        u = x[N * n * n:(N + 1) * n * n]
        out[name] = {"time_ms": round(t, 2), "converged": rc == binding.SMG_OK,
                     "newton_iterations": st["iterations"], "initial_solve_iterations": st["init_iterations"],
                     "inner_iterations": st["inner"],
                     "mean_inner_per_newton": round(float(np.mean(st["inner"])), 2) if st["inner"] else 0.0,
                     "step_lengths": st["gammas"], "phi": [float(f"{v:.3e}") for v in st["phi"]],
                     "ms_per_newton_step": round(t / max(st["iterations"], 1), 2),
                     "control_zero_fraction": round(float((u.abs() <= 1e-8).float().mean()), 4),
                     "control_at_bounds_fraction": round(float((u.abs() >= 50.0 - 1e-9).float().mean()), 4)}
    ctx.close()
    return out


def paper_tables(dev):
    """The settings of the paper's iteration-count tables on this library's grids
    (finite differences; the paper: P1 elements): the Gaussian-covariance field
    of eq. log_normal, y_d = exp(y^2) sin(2 pi x) sin(2 pi y), no source, damped
    collective Jacobi (theta 1/2) V(2,2), tolerance 1e-9.  Distributed control
    and the L^1 problem on the L-shape (N_h = 705 at 31x31, as printed), local
    control on the square (N_h = 961).  Defaults of the sub-tables: nu 1e-4,
    sigma^2 0.5, L^2 0.5 with M = 3 and 5^3 collocation nodes, 31x31 (three
    levels); the Monte Carlo sub-tables take sigma^2 1.5, L^2 0.1, M = 15.
    The linear-quadratic systems keep the printed rows of eq.
    full_space_optimality_system (rows="paper"), whose residual the printed
    stopping rule measures; the L^1 run the rescaled adjoint its Newton system
    is written in.  Counts beside the printed ones."""
    import numpy as np
    import torch
    from paper_2302_13680_amd import binding, inputs

    def problem(n=31, q=5, nu=1e-4, sigma2=0.5, L2=0.5, M=3, mc=None, rows="paper", **kw):
        common = dict(sigma=float(np.sqrt(sigma2)), decay=True, yd=inputs.paper_target(n), f=0.0,
                      field="gaussian", corr_len2=L2, rows=rows)
        if mc:
            return inputs.make_problem(n, mc, nu, M=M, seed=17, **common, **kw)
        return inputs.collocation_problem(n, q, nu, M=M, **common, **kw)

    def counts(p):
        ctx, f = binding.context_from_problem(p, device=dev, gmres_restart=30, theta=0.5,
                                              flags=binding.SMG_FLAG_JACOBI)
        x = torch.zeros(p.dof, dtype=torch.float64, device=dev)
        _, sv = timed_solve(ctx, x, f, binding.SMG_VCYCLE, 1e-9, maxit=300)
        _, sg = timed_solve(ctx, x, f, binding.SMG_GMRES, 1e-9, maxit=300)
        ctx.close()
        return [sv["iterations"], sg["iterations"]]

    def counts_or_stall(p, maxit=100):
        """counts(), a V-cycle that stalls reported as "stall (relres after maxit)"."""
        ctx, f = binding.context_from_problem(p, device=dev, gmres_restart=30, theta=0.5,
                                              flags=binding.SMG_FLAG_JACOBI)
        res = []
        for method in (binding.SMG_VCYCLE, binding.SMG_GMRES):
            x = torch.zeros(p.dof, dtype=torch.float64, device=dev)
            rc, st = ctx.solve(x, f, method, rtol=1e-9, maxit=maxit)
            res.append(st["iterations"] if rc == binding.SMG_OK else "stall (%.1e after %d)" % (st["relres"], maxit))
        ctx.close()
        return res

    out = {"field": "Gaussian covariance (eq. log_normal)", "smoother": "collective Jacobi theta 1/2, V(2,2)",
           "tol": 1e-9, "rows": "as printed (eq. full_space_optimality_system)",
           "format": "[V-cycles, GMRES] (this library) beside [printed]"}
    L = dict(domain="lshape")
    t1 = {}
    t1["nu"] = [{"nu": nu, "counts": counts(problem(nu=nu, **L)), "paper": pr}
                for nu, pr in ((1e-2, [18, 11]), (1e-4, [19, 13]), (1e-6, [19, 15]), (1e-8, [19, 15]))]
    t1["sigma2"] = [{"sigma2": s2, "counts": counts(problem(sigma2=s2, **L)), "paper": pr}
                    for s2, pr in ((0.1, [19, 13]), (0.5, [19, 13]), (1.0, [20, 13]), (1.5, [20, 13]))]
    t1["mesh"] = [{"n": n, "nodes": nh, "counts": counts(problem(n=n, **L)), "paper": pr}
                  for n, nh, pr in ((15, 161, [19, 13]), (31, 705, [19, 13]), (63, 2945, [20, 13]))]
    t1["N_collocation"] = [{"N": q ** 3, "counts": counts(problem(q=q, **L)), "paper": [19, 13]} for q in (2, 3, 4, 5)]
    t1["N_monte_carlo"] = [{"N": N, "counts": counts(problem(mc=N, sigma2=1.5, L2=0.1, M=15, **L)), "paper": pr}
                           for N, pr in ((100, [22, 16]), (500, [22, 15]), (1000, [22, 15]), (2000, [22, 15]))]
    out["distributed_lshape"] = t1
    R = dict(control_region=(0.25, 0.75, 0.25, 0.75))

    def counts_galerkin(p):
        """The control region as node factors of D_j and E_j coarsened by full
        weighting (the row-lumped Galerkin product R diag(m) P of the paper's
        Galerkin coarse operators) instead of the injected control mask."""
        t = (np.arange(p.n) + 1.0) / (p.n + 1)
        X, Y = np.meshgrid(t, t)
        eps = 1e-12
        m = ((X >= 0.25 - eps) & (X <= 0.75 + eps) & (Y >= 0.25 - eps) & (Y <= 0.75 + eps)).astype(np.float64)
        md = torch.tensor(m, dtype=torch.float64, device=dev)
        ctx, f = binding.context_from_problem(p, device=dev, gmres_restart=30, theta=0.5,
                                              flags=binding.SMG_FLAG_JACOBI)
        ctx.set_node_factors(md, md, binding.SMG_COARSEN_FULL)
        x = torch.zeros(p.dof, dtype=torch.float64, device=dev)
        _, sv = timed_solve(ctx, x, f, binding.SMG_VCYCLE, 1e-9, maxit=300)
        _, sg = timed_solve(ctx, x, f, binding.SMG_GMRES, 1e-9, maxit=300)
        ctx.close()
        return [sv["iterations"], sg["iterations"]]

    t2 = {"coarse_control": "counts: node factors by full weighting (Galerkin, row-lumped); "
                            "counts_injection: the injected control mask"}
    t2["nu"] = [{"nu": nu, "counts": counts_galerkin(problem(nu=nu)), "counts_injection": counts(problem(nu=nu, **R)),
                 "paper": pr}
                for nu, pr in ((1e-2, [17, 11]), (1e-4, [20, 13]), (1e-6, [26, 16]), (1e-8, [26, 18]))]
    t2["N_monte_carlo"] = [{"N": N, "counts": counts_galerkin(problem(mc=N, sigma2=1.5, L2=0.1, M=15)),
                            "counts_injection": counts(problem(mc=N, sigma2=1.5, L2=0.1, M=15, **R)), "paper": pr}
                           for N, pr in ((100, [20, 14]), (1000, [21, 15]), (2000, [21, 14]))]
    out["local_square"] = t2

    def bproblem(n=63, q=5, nu=1e-4, sigma2=0.5, L2=0.5, M=3, mc=None):
        common = dict(sigma=float(np.sqrt(sigma2)), decay=True, field="gaussian", corr_len2=L2, rows="paper")
        if mc:
            return inputs.boundary_control_problem(n, mc, nu, M=M, seed=17, **common)
        return inputs.boundary_collocation_problem(n, q, nu, M=M, **common)
    t3 = {"construction": "reflection across Gamma: a domain and a control on the mirror row, "
                          "control blocks x2 per coarsening"}
    t3["nu"] = [{"nu": nu, "counts": counts_or_stall(bproblem(nu=nu)), "paper": pr}
                for nu, pr in ((1e-2, [17, 14]), (1e-4, [22, 15]), (1e-6, [23, 17]), (1e-8, [21, 16]))]
    t3["sigma2"] = [{"sigma2": s2, "counts": counts(bproblem(sigma2=s2)), "paper": pr}
                    for s2, pr in ((0.1, [16, 13]), (0.5, [17, 14]), (1.0, [17, 14]), (1.5, [17, 14]))]
    t3["mesh"] = [{"nodes": nh, "counts": counts(bproblem(n=n)), "paper": pr}
                  for n, nh, pr in ((31, 240, [16, 12]), (63, 992, [17, 14]), (127, 4032, [21, 16]))]
    t3["N_collocation"] = [{"N": q ** 3, "counts": counts(bproblem(q=q)), "paper": pr}
                           for q, pr in ((2, [16, 13]), (3, [17, 14]), (4, [17, 14]), (5, [17, 14]))]
    t3["N_monte_carlo"] = [{"N": N, "counts": counts(bproblem(mc=N, sigma2=1.5, L2=0.1, M=15)), "paper": pr}
                           for N, pr in ((100, [18, 15]), (1000, [19, 16]), (2000, [20, 16]))]
    out["boundary_control"] = t3
    p = problem(rows="scaled", **L)
    ctx, f = binding.context_from_problem(p, device=dev, gmres_restart=30, theta=0.5, flags=binding.SMG_FLAG_JACOBI,
                                          ssn=True)
    x = torch.zeros(p.dof, dtype=torch.float64, device=dev)
    l1 = {"nu": 1e-4, "beta": 1e-2, "box": [-50.0, 50.0], "domain": "L-shape, 705 nodes",
          "paper_newton_vcycle_gmres": [5, 22.6, 14.2]}
    for name, method in (("gmres", binding.SMG_GMRES), ("vcycle", binding.SMG_VCYCLE)):
        prm = binding.ssn_params(1e-4, 1e-2, -50.0, 50.0, (1.0 / 32) ** 2, inner_method=method)
        _, rc, st = ssn_run(ctx, x, f, prm)
        l1[name + "_newton"] = st["iterations"]
        l1[name + "_mean_inner"] = round(float(np.mean(st["inner"])), 2) if st["inner"] else 0.0
        l1[name + "_converged"] = rc == binding.SMG_OK
    ctx.close()
    out["l1_semismooth_newton_lshape"] = l1
    return out


def ssn_tables(dev):
    """The settings of the paper's L^1 tables (Section 5) on the L-shape with the
    Gaussian field, collocation nodes and the Jacobi-smoothed V-cycle: Newton
    iterations and the mean V-cycle and GMRES iterations per Newton system
    (merit 1e-9, systems 1e-11), beside the printed [Newton, V-cycles, GMRES].
    Defaults: 31x31 (705 nodes), 5^3 nodes, sigma^2 0.5, L^2 0.5, nu 1e-4,
    beta 1e-2, -50 <= u <= 50.  The nu sweep runs from u = 0 and by continuation
    (each nu = 10^-j, j = 2..8, started from the control of the previous one)."""
    import numpy as np
    import torch
    from paper_2302_13680_amd import binding, inputs

    def problem(n=31, q=5, nu=1e-4, sigma2=0.5):
        return inputs.collocation_problem(n, q, nu, M=3, sigma=float(np.sqrt(sigma2)), decay=True,
                                          yd=inputs.paper_target(n), f=0.0, field="gaussian", corr_len2=0.5,
                                          domain="lshape")

    def run(p, beta=1e-2, u0=None, methods=("gmres", "vcycle")):
        ctx, f = binding.context_from_problem(p, device=dev, gmres_restart=30, theta=0.5,
                                              flags=binding.SMG_FLAG_JACOBI, ssn=True)
        x = torch.zeros(p.dof, dtype=torch.float64, device=dev)
        res = {}
        nn = p.n * p.n
        for name in methods:
            method = binding.SMG_GMRES if name == "gmres" else binding.SMG_VCYCLE
            prm = binding.ssn_params(p.nu, beta, -50.0, 50.0, (1.0 / (p.n + 1)) ** 2, inner_method=method,
                                     maxit=100)
            x.zero_()
            if u0 is not None:
                x[p.N * nn:(p.N + 1) * nn] = u0
            rc, st = ctx.ssn_solve(x, f, prm)
            res[name] = [st["iterations"], round(float(np.mean(st["inner"])), 1) if st["inner"] else 0.0,
                         rc == binding.SMG_OK]
        u = x[p.N * nn:(p.N + 1) * nn].clone()
        ctx.close()
        return res, u

    def row(key, val, p, printed, beta=1e-2):
        r, _ = run(p, beta)
        return {key: val, "gmres [newton, mean its, converged]": r["gmres"],
                "vcycle [newton, mean its, converged]": r["vcycle"], "paper": printed}

    out = {"domain": "L-shape, 705 nodes at 31x31", "smoother": "collective Jacobi theta 1/2, V(2,2)"}
    out["sigma2"] = [row("sigma2", s2, problem(sigma2=s2), pr) for s2, pr in
                     ((0.1, [4, 22.5, 14]), (0.5, [5, 22.6, 14.2]), (1.0, [8, 23.0, 11.8]), (1.5, [14.9, 22.9, 15.0]))]
    out["mesh"] = [row("nodes", nh, problem(n=n), pr) for n, nh, pr in
                   ((15, 161, [5, 22.0, 15.2]), (31, 705, [5, 22.6, 14.2]), (63, 2945, [5, 22.2, 14.0]))]
    out["N_collocation"] = [row("N", q ** 3, problem(q=q), pr) for q, pr in
                            ((2, [5, 21.0, 13.0]), (3, [5, 21.6, 14.0]), (4, [5, 22.0, 14.0]), (5, [5, 22.6, 14.2]))]
    out["beta"] = [row("beta", b, problem(), pr, beta=b) for b, pr in
                   ((0.0, [4, 22.5, 14.8]), (1e-4, [4, 22.5, 14.5]), (1e-3, [5, 22.4, 14.8]), (1e-2, [5, 22.6, 14.2]))]
    out["nu_from_zero"] = [row("nu", nu, problem(nu=nu), pr) for nu, pr in
                           ((1e-2, [2, 23.0, 14.5]), (1e-4, [5, 22.7, 14.2]), (1e-6, [17, 25.6, 15.0]),
                            (1e-8, [50, 41.4, 17.2]))]
    printed_cont = {1e-2: [2, 23.0, 14.5], 1e-4: [4, 22.7, 14.2], 1e-6: [5, 22.25, 15.4], 1e-8: [8, 58.8, 20.9]}
    cont, u = [], None
    for j in range(2, 9):
        nu = 10.0 ** -j
        r, u = run(problem(nu=nu), u0=u, methods=("gmres",))
        if nu in printed_cont:
            cont.append({"nu": nu, "gmres [newton, mean its, converged]": r["gmres"], "paper": printed_cont[nu]})
    out["nu_continuation"] = cont
    return out


def cvar_problem(n=31, N=500, seed=23):
    """The risk-averse table's problem: L-shape, Gaussian field sigma^2 1, L^2 0.1,
    15 modes, Monte Carlo samples, nu 1e-4, the paper's target, f = 0."""
    from paper_2302_13680_amd import inputs
    return inputs.make_problem(n, N, 1e-4, M=15, sigma=1.0, seed=seed, yd=inputs.paper_target(n), f=0.0,
                               field="gaussian", corr_len2=0.1, domain="lshape")


def cvar_run(dev, p, lam, eps, x=None, t0=0.0):
    """Algorithm 3 on problem p (GMRES(30) with the Jacobi V-cycle): returns x,
    the solver's stats and a table row with the device wall time."""
    import numpy as np
    import torch
    from paper_2302_13680_amd import binding
    ctx, f = binding.context_from_problem(p, device=dev, gmres_restart=30, theta=0.5,
                                          flags=binding.SMG_FLAG_JACOBI | binding.SMG_FLAG_CVAR)
    mass = -float(p.d[0])
    zeta = np.asarray(p.c) / mass
    live = np.ones(p.n * p.n) if p.domain is None else np.asarray(p.domain).reshape(-1)
    yd = torch.tensor((np.asarray(p.yd).reshape(-1) * live).reshape(p.n, p.n), dtype=torch.float64, device=dev)
    if x is None:
        x = torch.zeros(p.dof, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    rc, st = ctx.cvar_solve(x, f, yd, zeta, lam, eps, mass, t0=t0)
    torch.cuda.synchronize()
    wall = 1e3 * (time.perf_counter() - t_start)
    ctx.close()
    mean = st["linear_total"] / max(st["linear_solves"], 1)
    row = {"counts": [st["outer"], st["inner_total"], round(mean, 1)], "inner_capped": st["inner_capped"],
           "inner_stalled": st["inner_stalled"],
           "converged": rc == binding.SMG_OK,
           "t": st["t"], "wall_ms": round(wall, 1)}
    print("cvar", p.n, p.N, lam, eps, json.dumps(row), file=sys.stderr, flush=True)
    return x, st, row


def cvar_tables(dev):
    """The settings of the paper's risk-averse table (Section 6, Algorithm 3) on
    the L-shape with the Gaussian field (sigma^2 1, L^2 0.1, 15 modes), Monte
    Carlo samples, nu 1e-4 and the Jacobi-smoothed V-cycle inside GMRES(30):
    [outer Newton, inner Newton, mean GMRES iterations per system] beside the
    printed [outer, inner, mean V-cycles, mean GMRES]; the eps sweep continues
    from the previous eps's solution (x and t), as the paper does.  Wall time of
    every run on the device."""
    problem = cvar_problem

    def run(p, lam, eps, x=None, t0=0.0):
        return cvar_run(dev, p, lam, eps, x=x, t0=t0)

    out = {"method": "GMRES(30), one V-cycle of S(c) as preconditioner, rank-one terms in the operator",
           "inner_rule": "printed: max(||F_1||/||F_1(x^0)||, ||F_1||) <= 1e-8, Newton steps backtracking on "
                         "||F_1||, at most 50; inner_stalled counts evaluations that ended at the rounding floor "
                         "(no decrease with ||F_1|| <= 1e-8), inner_capped those that ended at the cap",
           "format": "[outer, inner Newton, mean GMRES] (this library) beside [outer, inner, mean V-cycles, mean GMRES]"}
    out["mesh"] = []
    for n, nh, pr in ((15, 161, [5, 62, 23.0, 13.9]), (31, 705, [6, 79, 28.0, 15.5]), (63, 2945, [6, 79, 26.2, 14.8])):
        _, _, r = run(problem(n=n), 0.9, 1e-2)
        out["mesh"].append(dict(nodes=nh, **r, paper=pr))
    out["N"] = []
    for N, pr in ((500, [6, 63, 55.4, 17.5]), (1000, [5, 66, 24.4, 14.0]), (2000, [4, 51, 24.4, 14.0])):
        _, _, r = run(problem(N=N), 0.95, 1e-2)
        out["N"].append(dict(N=N, **r, paper=pr))
    out["lambda"] = []
    for lam, pr in ((0.0, [0, 1, 21.0, 14.0]), (0.5, [5, 21, 19.4, 13.6]), (0.95, [5, 64, 23.2, 13.8]),
                    (0.99, [8, 129, 33.4, 17.5])):
        _, _, r = run(problem(N=2000), lam, 1e-2)
        out["lambda"].append(dict(lam=lam, **r, paper=pr))
    out["eps_continuation"] = []
    p = problem(N=1000)
    x, t = None, 0.0
    for eps, pr in ((1e-1, [7, 67, 22.5, 17.0]), (1e-2, [3, 42, 29.1, 14.8]), (1e-3, [2, 20, None, 27.9]),
                    (1e-4, [1, 15, 58.0, 55.6])):
        x, st, r = run(p, 0.95, eps, x=x, t0=t)
        t = st["t"]
        out["eps_continuation"].append(dict(eps=eps, **r, paper=pr))
    return out


def sweep_bytes(n: int, N: int, word: int) -> float:
    """Algorithmic bytes of one red+black sweep: per node-sample y, p, the two
    right-hand sides and the two face arrays read once and y, p written once (8
    words), per node u and f_U (2 words)."""
    return float((8 * N + 2) * n * n * word)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_oracle_sample(prob, budget_s: float = 10.0, max_cycles: int = 3):
    """The FP64 CPU oracle on the same instance: V(2,2) cycles from zero until
    budget_s has elapsed (at least one), setup excluded.  Returns the record."""
    import numpy as np
    from oracle import oracle as orc
    o = orc.Oracle(prob)
    fp = prob.rhs_paper()
    x = np.zeros(o.vlen())
    cycles, t = 0, 0.0
    while cycles < max_cycles and (cycles == 0 or t < budget_s):
        t0 = time.perf_counter()
        x = o.vcycle(x, fp, 1)
        t += time.perf_counter() - t0
        cycles += 1
    return {"value": round(prob.dof * 4 * cycles / t, 1), "unit": "DoF-sweeps/s",
            "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"{cycles} V(2,2) cycles of the FP64 oracle from zero on the same instance "
                      f"({t:.1f} s, setup excluded)",
            "cpu": cpu_model()}


def time_sweep(ctx, xa, xb, f, stream, launches, fp32=False):
    """Average duration (us) of `launches` finest-level one-launch sweeps
    (alternating between xa and xb), HIP events on the library's stream."""
    import torch
    sweep = ctx.sweep32 if fp32 else ctx.sweep
    for i in range(4):
        sweep(0, xa, xb, f) if i % 2 == 0 else sweep(0, xb, xa, f)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(launches):
        sweep(0, xa, xb, f) if i % 2 == 0 else sweep(0, xb, xa, f)
    e1.record(stream)
    e1.synchronize()
    return 1e3 * e0.elapsed_time(e1) / launches


def roofline_sweep(ctx, f, n, N, dev, launches, traffic_kind):
    """The dominant kernel of the FP64 solve: the finest-level sweep.  Where the
    level takes the one-launch sweep (k_sweep_fused) one launch is a whole
    red+black sweep, priced at its algorithmic bytes (8 words per node-sample,
    2 per node); else the half-sweep at half of them.  Average launch duration
    from HIP events on the library's stream."""
    import torch
    xa = torch.zeros(ctx.vlen(), dtype=torch.float64, device=dev)
    xb = torch.empty_like(xa)
    one = ctx.sweep(0, xa, xb, f)
    if one:
        us = time_sweep(ctx, xa, xb, f, ctx.stream, launches)
        algo = sweep_bytes(n, N, 8)
        kernel = (f"k_sweep_fused<double,4,{2 if N % 2 == 0 else 1},kPlain,all> finest level "
                  "(red+black sweep, every field written)")
    else:
        us = time_halfsweep(ctx, xa, f, ctx.stream, launches)
        algo, kernel = sweep_bytes(n, N, 8) / 2, "k_halfsweep<double,64,4> finest level"
    achieved = algo / (us * 1e-6) / 1e9
    del xa, xb
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(traffic_kind),
            "kernel": kernel, "avg_launch_us": round(us, 2), "bytes_per_launch": algo}


def stream_copy_gbs(dev):
    """Achievable-bandwidth reference: the library's streaming copy, 1 GiB each way."""
    import torch
    from paper_2302_13680_amd import binding
    ca = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    cb = torch.empty_like(ca)
    for _ in range(3):
        binding.stream_copy(cb, ca)
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(10):
        binding.stream_copy(cb, ca)
    c1.record()
    c1.synchronize()
    gbs = 2 * ca.numel() * 8 / (c0.elapsed_time(c1) / 10 * 1e-3) / 1e9
    del ca, cb
    return round(gbs, 1)


def medium_section(dev, args):
    """255x255, N=64 (FP64): GMRES(30) and stationary V(2,2) to 1e-8 and 1e-10,
    the Jacobi smoother, collocation, local control and the semismooth Newton
    method on the same grid.  The working set (~0.2 GB) stays in the 256 MB
    Infinity Cache, so the bandwidth figures here are not HBM figures."""
    import torch
    from paper_2302_13680_amd import binding, inputs
    prob = inputs.medium_fp64()
    n, N, dof = prob.n, prob.N, prob.dof
    ctx, f = binding.context_from_problem(prob, device=dev, gmres_restart=30)
    x = torch.zeros(dof, dtype=torch.float64, device=dev)
    out = {"section": "medium_fp64", "workload": "255x255, N=64, 6 KL modes a_m=0.5/m, nu=1e-4, FP64",
           "infinity_cache_resident": True}
    for name, method, rtol in (("gmres30", binding.SMG_GMRES, 1e-8), ("vcycle", binding.SMG_VCYCLE, 1e-8),
                               ("gmres30_1e-10", binding.SMG_GMRES, 1e-10)):
        timed_solve(ctx, x, f, method, rtol)
        ts = []
        for _ in range(3):
            t, st = timed_solve(ctx, x, f, method, rtol)
            ts.append(t)
        out[name] = {"time_ms": round(sorted(ts)[1], 3), "iterations": st["iterations"],
                     "vcycles": st["inner_iterations"] if method == binding.SMG_GMRES else st["iterations"]}
    us = time_halfsweep(ctx, torch.zeros(dof, dtype=torch.float64, device=dev), f, ctx.stream, 200)
    out["finest_halfsweep_us"] = round(us, 2)
    out["finest_halfsweep_rate_GBs_at_sweep_bytes"] = round(sweep_bytes(n, N, 8) / 2 / (us * 1e-6) / 1e9, 1)
    cj = binding.Context(n, N, ctx.kx, ctx.ky, prob.c, prob.d, prob.e, prob.g, gmres_restart=30, theta=0.5,
                         flags=binding.SMG_FLAG_JACOBI)
    jac = {"smoother": "damped collective Jacobi, theta=0.5, V(2,2)"}
    for name, method in (("gmres30", binding.SMG_GMRES), ("vcycle", binding.SMG_VCYCLE)):
        timed_solve(cj, x, f, method, 1e-8)
        t, stj = timed_solve(cj, x, f, method, 1e-8)
        jac[name + "_time_to_1e-8_ms"] = round(t, 3)
        jac[name + "_iterations"] = stj["iterations"]
    cj.close()
    out["jacobi_smoother"] = jac
    psc = inputs.collocation_problem(n, 4, 1e-4, M=3, sigma=0.5, decay=True)
    csc, fsc = binding.context_from_problem(psc, device=dev, gmres_restart=30)
    xsc = torch.zeros(psc.dof, dtype=torch.float64, device=dev)
    sc = {"samples": "tensor Gauss-Hermite, M=3 variables, 4 points each (N=64), weights zeta_j"}
    for name, method in (("gmres30", binding.SMG_GMRES), ("vcycle", binding.SMG_VCYCLE)):
        timed_solve(csc, xsc, fsc, method, 1e-8)
        t, stc = timed_solve(csc, xsc, fsc, method, 1e-8)
        sc[name + "_time_to_1e-8_ms"] = round(t, 3)
        sc[name + "_iterations"] = stc["iterations"]
    csc.close()
    out["stochastic_collocation"] = sc
    plc = inputs.make_problem(n, N, 1e-4, M=6, sigma=0.5, decay=True, seed=1,
                              control_region=(0.25, 0.75, 0.25, 0.75))
    clc, flc = binding.context_from_problem(plc, device=dev, gmres_restart=30)
    xlc = torch.zeros(plc.dof, dtype=torch.float64, device=dev)
    lc = {"control": "on the nodes of [0.25, 0.75]^2 only (control mask)"}
    for name, method in (("gmres30", binding.SMG_GMRES), ("vcycle", binding.SMG_VCYCLE)):
        timed_solve(clc, xlc, flc, method, 1e-8)
        t, stl = timed_solve(clc, xlc, flc, method, 1e-8)
        lc[name + "_time_to_1e-8_ms"] = round(t, 3)
        lc[name + "_iterations"] = stl["iterations"]
    clc.close()
    out["local_control"] = lc
    ctx.close()
    out["semismooth_newton"] = ssn_section(dev, n, N, args)
    return out


def emit(rec):
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sweeps", type=int, default=60, help="sweep launches timed for the roofline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--quick", action="store_true", help="the headline workload only")
    ap.add_argument("--large-only", action="store_true",
                    help="run only the 511x511, N=256 mixed-precision section (for profiling)")
    ap.add_argument("--medium-gmres-only", action="store_true",
                    help="run only 4 FP64 GMRES(30) solves of the 255x255, N=64 instance (for tracing)")
    ap.add_argument("--cvar-only", action="store_true",
                    help="run only the risk-averse solver at 705 nodes, N=2000, lambda 0.95 (for profiling)")
    ap.add_argument("--tune-cache", default=os.path.join(tempfile.gettempdir(), "smg_autotune_lanes.json"))
    ap.add_argument("--counters", nargs="?", const="medium", choices=["medium", "large"],
                    help="launch only the finest-level FP64 passes of the 255x255, N=64 (medium) or "
                         "511x511, N=256 (large) workload (20 sweeps, 5 residuals, 5 residual + "
                         "restrictions, 2 V-cycles) and a 1 GiB device copy (5x), for hardware-counter passes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU only; multi-GPU sharding is a design "
                                   "note, not an implemented path", "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    from paper_2302_13680_amd import binding, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.cvar_only:
        p = cvar_problem(31, 2000)
        cvar_run(dev, p, 0.95, 1e-2)                 # warm-up (graph capture)
        _, _, row = cvar_run(dev, p, 0.95, 1e-2)
        emit({"cvar": dict(workload="L-shape 705 nodes, N=2000, lambda 0.95, eps 1e-2", **row)})
        return
    if args.large_only:
        large, _, _, _ = large_mixed_section(dev)
        emit({"large_mixed": large})
        return
    if args.medium_gmres_only:
        prob = inputs.medium_fp64()
        ctx, f = binding.context_from_problem(prob, device=dev, gmres_restart=30)
        x = torch.zeros(prob.dof, dtype=torch.float64, device=dev)
        timed_solve(ctx, x, f, binding.SMG_GMRES, 1e-8)             # warm-up (graph capture)
        runs = [timed_solve(ctx, x, f, binding.SMG_GMRES, 1e-8) for _ in range(3)]
        emit({"medium_gmres": {"workload": "255x255, N=64, FP64 GMRES(30) + V(2,2) to 1e-8",
                               "time_ms": [round(t, 3) for t, _ in runs],
                               "iterations": runs[-1][1]["iterations"]}})
        return
    if args.counters:
        prob = inputs.large_mixed() if args.counters == "large" else inputs.medium_fp64()
        ctx, f = binding.context_from_problem(prob, device=dev, gmres_restart=0)
        x = torch.zeros(prob.dof, dtype=torch.float64, device=dev)
        halfsweep_counter_run(ctx, x, f, prob.n, prob.N)
        return

    # ---------------- headline: 511x511, N=256, FP64 GMRES(30) + V(2,2) to 1e-8
    prob = inputs.large_mixed()
    n, N, dof = prob.n, prob.N, prob.dof
    ctx, f = binding.context_from_problem(prob, device=dev, gmres_restart=30)
    levels = list(ctx.levels_n)
    x = torch.zeros(dof, dtype=torch.float64, device=dev)

    def solve(method, rtol):
        x.zero_()
        rc, st = ctx.solve(x, f, method, rtol=rtol, maxit=200, history=0)
        if rc != binding.SMG_OK:
            raise RuntimeError(f"solve did not converge: {st}")
        return st

    for _ in range(args.warmup):
        solve(binding.SMG_GMRES, args.rtol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles = 0
    for _ in range(args.steps):
        st = solve(binding.SMG_GMRES, args.rtol)
        cycles += st["inner_iterations"]
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    ms_per_step = 1e3 * t_total / args.steps
    value = dof * 4 * cycles / t_total
    gmres_its = st["iterations"]

    # the plain FP64 stationary V-cycle on the same GPU (the comparison baseline)
    tv = []
    for i in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stv = solve(binding.SMG_VCYCLE, args.rtol)
        torch.cuda.synchronize()
        if i:
            tv.append(1e3 * (time.perf_counter() - t0))
    t_vcycle_ms = sorted(tv)[1]
    roofline = roofline_sweep(ctx, f, n, N, dev, args.sweeps, "sweep_f64_large")
    ctx.close()
    del ctx, x
    torch.cuda.empty_cache()
    roofline["stream_copy_GBs"] = stream_copy_gbs(dev)

    # FP32 smoother, residual and transfers inside FP64 refinement (FGMRES(30) and stationary)
    c32 = binding.Context(n, N, torch.from_numpy(prob.faces_node()[0]).to(dev),
                          torch.from_numpy(prob.faces_node()[1]).to(dev), prob.c, prob.d, prob.e, prob.g,
                          gmres_restart=30, precision=binding.SMG_F32)
    x = torch.zeros(dof, dtype=torch.float64, device=dev)
    mixed = {}
    for name, method in (("fgmres30", binding.SMG_GMRES), ("vcycle", binding.SMG_VCYCLE)):
        timed_solve(c32, x, f, method, args.rtol)
        ts = []
        for _ in range(3):
            t, st32 = timed_solve(c32, x, f, method, args.rtol)
            ts.append(t)
        mixed[name] = (round(sorted(ts)[1], 2), st32["iterations"], st32["inner_iterations"])
    c32.close()
    del c32, x, f
    torch.cuda.empty_cache()

    # ---------------- further sections, one JSON line each
    failed = []
    if not args.quick:
        def run_section(name, fn):
            try:
                rec = fn()
                rec.setdefault("section", name)
                emit(rec)
            except Exception as exc:   # a failing section is reported, the headline still printed
                failed.append(name)
                emit({"section": name, "error": repr(exc)})
            torch.cuda.empty_cache()

        def large():
            rec, c32b, fl, xl = large_mixed_section(dev)
            del c32b, fl, xl
            return rec
        run_section("large_mixed", large)
        run_section("medium_fp64", lambda: medium_section(dev, args))
        run_section("large_semismooth_newton", lambda: large_ssn_section(dev))
        run_section("batch", lambda: batch_section(dev, args.tune_cache))
        run_section("learned", lambda: learned_section(dev))

        def paper():
            rec = paper_tables(dev)
            rec["l1_tables"] = ssn_tables(dev)
            rec["cvar_tables"] = cvar_tables(dev)
            return rec
        run_section("paper_settings", paper)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_oracle_sample(prob)

    emit({
        "metric": METRIC, "value": round(value, 1), "unit": "DoF-sweeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "LQ-OCPUU 511x511 grid, N=256 samples, 6 KL modes a_m=1.0/m, nu=1e-4; "
                               "FP64 GMRES(30) + V(2,2) red-black collective GS to rel. residual 1e-8",
                   "dof": dof, "levels": levels},
        "time_to_1e-8_ms": round(ms_per_step, 2), "gmres_iterations": gmres_its,
        "fp64_vcycle_time_to_1e-8_ms": round(t_vcycle_ms, 2), "fp64_vcycle_cycles": stv["iterations"],
        "fp32_refined_fgmres30_ms": mixed["fgmres30"][0], "fp32_refined_vcycle_ms": mixed["vcycle"][0],
        "roofline": roofline, "cpu_baseline": cpu, "sections_failed": failed,
    })


if __name__ == "__main__":
    main()
