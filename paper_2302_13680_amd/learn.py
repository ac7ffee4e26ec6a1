"""Learned warm start: data from the multigrid solver, training on the GPU with
the library's network kernels, evaluation against the zero start.

Data: each instance (seeded KL coefficients, nu log-uniform in [1e-5, 1e-3],
y_d a random sum of three sine products) is solved by the library to a
relative residual of 1e-8; the features (mean/std over samples of the node
log-coefficient, y_d, log10 nu + 4) and the fields (u, mean y, mean p) of the
solution are extracted by the library (smg_net_features / smg_net_targets).
Training: mean squared error of the per-channel standardized fields over the
interior nodes, Adam, mini-batches, every step in smg_net_train_step.
Evaluation: for held-out seeds, V-cycles and wall time to 1e-8 from the zero
start and from the lifted prediction x0 (smg_net_lift), inference at batch 1.
The warm start is checked against the zero start after one V-cycle: the warm solve goes on
from V(x0) when ||f - S V(x0)|| <= rho0 ||f||, where rho0 is the relative
residual one V-cycle from zero leaves (the median over the training solves);
otherwise it falls back to the zero-start solve (the checking cycle is counted).
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import binding, inputs


def grid_for(n: int) -> int:
    """Network grid: the instance's n x n nodes padded up to a multiple of 8."""
    return ((n + 1 + 7) // 8) * 8


def param_init(seed: int = 0) -> np.ndarray:
    """He-style initial weights (normal, variance 2 / fan-in), zero biases, in the
    parameter layout of the library (per layer W[cout][tap][cin] then b)."""
    arch = [(4, 16, 9), (16, 16, 9), (16, 32, 9), (32, 32, 9), (32, 48, 9), (48, 48, 9), (48, 48, 9),
            (48, 48, 9), (48, 48, 9), (48, 48, 9), (48, 32, 9), (32, 32, 9), (32, 16, 9), (16, 16, 9),
            (16, 3, 1)]
    rng = np.random.default_rng(seed)
    parts = []
    for (ci, co, t) in arch:
        parts.append(rng.standard_normal(co * t * ci) * math.sqrt(2.0 / (t * ci)))
        parts.append(np.zeros(co))
    theta = np.concatenate(parts)
    # small output layer: the initial prediction is close to the mean field
    nout = 3 * 16 + 3
    theta[-nout:] *= 0.1
    return theta.astype(np.float32)


class Instance:
    """One instance on the device with its solver context."""

    def __init__(self, seed: int, n: int, N: int, device, precision=binding.SMG_F64):
        nu, yd, xi = inputs.learned_instance_params(seed, n, N)
        kx, ky, f, c, d, e, g = inputs.make_problem_device(n, N, nu, xi, yd, device=device)
        self.n, self.N, self.nu, self.seed = n, N, nu, seed
        self.kx, self.ky, self.f = kx, ky, f
        self.ctx = binding.Context(n, N, kx, ky, c, d, e, g, gmres_restart=0, precision=precision)
        self.dof = (2 * N + 1) * n * n


def solve_time(inst, x, rtol=1e-8, maxit=100):
    """Zero start: x is cleared, then solved; returns (ms, stats, rc)."""
    import torch
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = inst.ctx.solve(x, inst.f, binding.SMG_VCYCLE, rtol=rtol, maxit=maxit, history=0)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0), st, rc


def make_dataset(seeds, n=127, N=128, device="cuda", log=None, first_cycle=None):
    """Solve every seed to 1e-8 and return (features, raw targets) as device tensors
    (S, H, H, 4) and (S, H, H, 3) (targets not yet standardized).  first_cycle (a
    list) receives each solve's relative residual after its first V-cycle."""
    import torch
    H = grid_for(n)
    S = len(seeds)
    feats = torch.zeros((S, H, H, 4), dtype=torch.float32, device=device)
    raw = torch.zeros((S, H, H, 3), dtype=torch.float32, device=device)
    ident = [0.0, 0.0, 0.0, 1.0, 1.0, 1.0]
    t0 = time.perf_counter()
    for i, s in enumerate(seeds):
        inst = Instance(s, n, N, device)
        x = torch.zeros(inst.dof, dtype=torch.float64, device=device)
        rc, st = inst.ctx.solve(x, inst.f, binding.SMG_VCYCLE, rtol=1e-8, maxit=100,
                                history=4 if first_cycle is not None else 0)
        if rc != binding.SMG_OK:
            raise RuntimeError(f"training solve {s} did not converge: {st}")
        if first_cycle is not None:
            first_cycle.append(st["history"][1] / st["history"][0])
        binding.net_features(inst.ctx, inst.f, H, feats[i])
        binding.net_targets(inst.ctx, x, H, ident, raw[i])
        # third field as N mean(p) / nu: the control row (f_U = 0, G = nu h^2 I,
        # D_j = -h^2 I) makes it equal to u, free of the 1/nu scale of mean(p)
        raw[i, :, :, 2] *= N / inst.nu
        inst.ctx.close()
        if log and (i + 1) % 250 == 0:
            log(f"dataset {i + 1}/{S} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return feats, raw


def standardization(raw, n):
    """Per-channel mean and standard deviation over the interior nodes."""
    v = raw[:, :n, :n, :].reshape(-1, 3).double()
    mean = v.mean(0)
    std = v.std(0).clamp_min(1e-30)
    return [float(m) for m in mean] + [float(s) for s in std]


def standardize(raw, norm, n):
    import torch
    mean = torch.tensor(norm[:3], dtype=raw.dtype, device=raw.device)
    std = torch.tensor(norm[3:], dtype=raw.dtype, device=raw.device)
    t = (raw - mean) / std
    t[:, n:, :, :] = 0.0
    t[:, :, n:, :] = 0.0
    return t.contiguous()


def train(net, feats, targets, n, epochs=20, lr=2e-3, seed=0, log=None, lr_final=2e-4):
    """Adam on mini-batches of net.B samples (the last partial batch is dropped);
    cosine decay of the learning rate from lr to lr_final.  Returns the loss per
    epoch (mean over its steps)."""
    import torch
    S = feats.shape[0]
    B = net.B
    rng = np.random.default_rng(seed)
    steps_per_epoch = S // B
    total = max(1, epochs * steps_per_epoch)
    xb = torch.empty((B,) + tuple(feats.shape[1:]), dtype=feats.dtype, device=feats.device)
    tb = torch.empty((B,) + tuple(targets.shape[1:]), dtype=targets.dtype, device=targets.device)
    hist = []
    step = 0
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(S), device=feats.device)
        acc = 0.0
        for b in range(steps_per_epoch):
            idx = perm[b * B:(b + 1) * B]
            torch.index_select(feats, 0, idx, out=xb)
            torch.index_select(targets, 0, idx, out=tb)
            cur = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * step / total))
            acc += net.train_step(xb, tb, n, cur)
            step += 1
        hist.append(acc / max(1, steps_per_epoch))
        if log:
            log(f"epoch {ep + 1}/{epochs} loss {hist[-1]:.4e}")
    return hist


def predict(net, feats):
    """Forward the network over (S, H, H, 4) features in mini-batches of net.B."""
    import torch
    S = feats.shape[0]
    B = net.B
    out = torch.empty(feats.shape[:3] + (3,), dtype=torch.float32, device=feats.device)
    xb = torch.zeros((B,) + tuple(feats.shape[1:]), dtype=feats.dtype, device=feats.device)
    ob = torch.empty((B,) + tuple(out.shape[1:]), dtype=torch.float32, device=feats.device)
    for s in range(0, S, B):
        m = min(B, S - s)
        xb.zero_()
        xb[:m] = feats[s:s + m]
        net.forward(xb, ob)
        out[s:s + m] = ob[:m]
    return out


def evaluate(net, seeds, norm, n=127, N=128, device="cuda", rtol=1e-8, rho0=None):
    """Warm start against zero start on held-out seeds, inference at batch 1 (a
    batch-1 copy of the trained network).  rho0: the zero start's relative
    residual after one V-cycle (median over the training solves; None: check
    ||f - S x0|| <= ||f|| before any cycle).  Returns per-seed records."""
    import torch
    H = grid_for(n)
    net1 = binding.Net(1, H, device=device)
    theta = torch.empty(net.np, dtype=torch.float32, device=device)
    net.get_params(theta)
    net1.set_params(theta)
    feat = torch.zeros((1, H, H, 4), dtype=torch.float32, device=device)
    pred = torch.empty((1, H, H, 3), dtype=torch.float32, device=device)
    recs = []
    truth = torch.empty((H, H, 3), dtype=torch.float32, device=device)
    ident = [0.0, 0.0, 0.0, 1.0, 1.0, 1.0]
    mean = torch.tensor(norm[:3], device=device)
    std = torch.tensor(norm[3:], device=device)
    for s in seeds:
        inst = Instance(s, n, N, device)
        x = torch.zeros(inst.dof, dtype=torch.float64, device=device)
        solve_time(inst, x, rtol)                       # warm-up: graph capture for (x, f)
        t_zero, st0, rc0 = solve_time(inst, x, rtol)
        # fields of the solution (third channel N mean(p) / nu, as in training)
        binding.net_targets(inst.ctx, x, H, ident, truth)
        truth[:, :, 2] *= N / inst.nu
        r = torch.empty_like(x)
        fnorm = float(torch.linalg.norm(inst.f))
        k = inst.nu / N                      # mean(p) = nu/N times the third field
        lift_norm = norm[:2] + [norm[2] * k] + norm[3:5] + [norm[5] * k]
        # warm start: features -> network -> lift -> one V-cycle -> check -> solve
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        binding.net_features(inst.ctx, inst.f, H, feat[0])
        net1.forward(feat, pred)
        binding.net_lift(inst.ctx, pred[0], H, lift_norm, x)
        torch.cuda.synchronize()
        t_inf = 1e3 * (time.perf_counter() - t0)
        rn0 = inst.ctx.residual(x, inst.f, r, norms=True)
        if rho0 is None:
            fell_back = not (rn0[0] <= fnorm)
            check_cycles = 0
            rel1 = None
        else:
            inst.ctx.vcycle(x, inst.f, 1)
            rn1 = inst.ctx.residual(x, inst.f, r, norms=True)
            rel1 = rn1[0] / fnorm
            fell_back = not (rel1 <= rho0)
            check_cycles = 1
        if fell_back:
            x.zero_()
        rc, st = inst.ctx.solve(x, inst.f, binding.SMG_VCYCLE, rtol=rtol, maxit=100, history=0)
        torch.cuda.synchronize()
        t_warm = 1e3 * (time.perf_counter() - t0)
        got = pred[0, :n, :n] * std + mean
        ref = truth[:n, :n]
        err = [float((torch.linalg.norm(got[..., c] - ref[..., c]) / torch.linalg.norm(ref[..., c])).item())
               for c in range(3)]
        err_mean = [float((torch.linalg.norm(mean[c] - ref[..., c]) / torch.linalg.norm(ref[..., c])).item())
                    for c in range(3)]
        # the lifted x0 without any rule: cycles and time from x0 (inference included)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        binding.net_lift(inst.ctx, pred[0], H, lift_norm, x)
        rc2, st2 = inst.ctx.solve(x, inst.f, binding.SMG_VCYCLE, rtol=rtol, maxit=100, history=0)
        torch.cuda.synchronize()
        t_lifted = 1e3 * (time.perf_counter() - t1)
        recs.append(dict(seed=s, nu=inst.nu, zero_cycles=st0["iterations"], zero_ms=t_zero,
                         warm_cycles=st["iterations"] + check_cycles, warm_ms=t_warm, fell_back=fell_back,
                         warm_cycles_no_fallback=st2["iterations"], warm_ms_no_fallback=t_inf + t_lifted,
                         inference_ms=t_inf, pred_rel_err=err, mean_pred_rel_err=err_mean,
                         x0_relres=rn0[0] / fnorm, relres_after_one_cycle=rel1, rho0=rho0,
                         converged=(rc == 0 and rc0 == 0 and rc2 == 0)))
        inst.ctx.close()
    net1.close()
    return recs


def summarize(recs):
    zc = np.array([r["zero_cycles"] for r in recs], dtype=float)
    wc = np.array([r["warm_cycles"] for r in recs], dtype=float)
    zt = np.array([r["zero_ms"] for r in recs])
    wt = np.array([r["warm_ms"] for r in recs])
    nf = np.array([r["warm_cycles_no_fallback"] for r in recs], dtype=float)
    return dict(instances=len(recs), zero_start_mean_cycles=float(zc.mean()),
                warm_start_no_fallback_mean_ms=float(np.mean([r["warm_ms_no_fallback"] for r in recs])),
                inference_mean_ms=float(np.mean([r["inference_ms"] for r in recs])),
                warm_start_no_fallback_mean_cycles=float(nf.mean()),
                warm_start_mean_cycles=float(wc.mean()), zero_start_mean_ms=float(zt.mean()),
                warm_start_mean_ms=float(wt.mean()),
                fallback_rate=float(np.mean([r["fell_back"] for r in recs])),
                median_x0_relres=float(np.median([r["x0_relres"] for r in recs])),
                median_relres_after_one_warm_cycle=(float(np.median([r["relres_after_one_cycle"] for r in recs]))
                                                    if recs and recs[0]["relres_after_one_cycle"] is not None
                                                    else None),
                rho0=recs[0]["rho0"] if recs else None,
                pred_rel_err_u_ybar_q=[float(np.mean([r["pred_rel_err"][c] for r in recs])) for c in range(3)],
                dataset_mean_rel_err_u_ybar_q=[float(np.mean([r["mean_pred_rel_err"][c] for r in recs]))
                                               for c in range(3)],
                all_converged=bool(all(r["converged"] for r in recs)))
