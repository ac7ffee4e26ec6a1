"""FP64 reference of the warm-start network (forward, backward, MSE loss, Adam).

TEST INFRASTRUCTURE ONLY.  Plain numpy, NHWC tensors, written from the
definitions: a 3x3 (or 1x1) convolution with zero padding is a sum over taps of
a pixel-wise matrix product; stride 2 samples every other output; "up" layers
read their input through a 2x nearest-neighbour upsampling; SiLU
a = z sigmoid(z).  Gradients follow the chain rule layer by layer; the test
suite checks them against central finite differences.

Network (4-level encoder-decoder, additive skips):
  idx  cin cout taps stride up  skip  act
   0    4   16   9    1     0   -     silu
   1   16   16   9    1     0   -     silu   -> skip 1
   2   16   32   9    2     0   -     silu
   3   32   32   9    1     0   -     silu   -> skip 3
   4   32   48   9    2     0   -     silu
   5   48   48   9    1     0   -     silu   -> skip 5
   6   48   48   9    2     0   -     silu
   7   48   48   9    1     0   -     silu
   8   48   48   9    1     1   5     silu
   9   48   48   9    1     0   -     silu
  10   48   32   9    1     1   3     silu
  11   32   32   9    1     0   -     silu
  12   32   16   9    1     1   1     silu
  13   16   16   9    1     0   -     silu
  14   16    3   1    1     0   -     none
Weights W_l: (cout, taps, cin), tap = 3 ky + kx; bias b_l: (cout,).
"""
from __future__ import annotations

import numpy as np

ARCH = [
    # cin, cout, taps, stride, up, skip, act
    (4, 16, 9, 1, 0, -1, 1),
    (16, 16, 9, 1, 0, -1, 1),
    (16, 32, 9, 2, 0, -1, 1),
    (32, 32, 9, 1, 0, -1, 1),
    (32, 48, 9, 2, 0, -1, 1),
    (48, 48, 9, 1, 0, -1, 1),
    (48, 48, 9, 2, 0, -1, 1),
    (48, 48, 9, 1, 0, -1, 1),
    (48, 48, 9, 1, 1, 5, 1),
    (48, 48, 9, 1, 0, -1, 1),
    (48, 32, 9, 1, 1, 3, 1),
    (32, 32, 9, 1, 0, -1, 1),
    (32, 16, 9, 1, 1, 1, 1),
    (16, 16, 9, 1, 0, -1, 1),
    (16, 3, 1, 1, 0, -1, 0),
]


def n_params():
    return sum(co * t * ci + co for (ci, co, t, *_r) in ARCH)


def unflatten(theta):
    """Flat parameter vector (per layer W then b) -> list of (W, b)."""
    out, o = [], 0
    for (ci, co, t, *_r) in ARCH:
        W = theta[o:o + co * t * ci].reshape(co, t, ci); o += co * t * ci
        b = theta[o:o + co]; o += co
        out.append((W, b))
    return out


def bf16_round(a):
    """Round float64/float32 values to bfloat16 (round to nearest even) and back."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def conv(x, W, b, stride, up):
    """z[b, y, x, co] = b[co] + sum_tap sum_ci W[co, tap, ci] in[b, y', x', ci]."""
    if up:
        x = x.repeat(2, axis=1).repeat(2, axis=2)
    taps = W.shape[1]
    k = 3 if taps == 9 else 1
    pad = k // 2
    B, H, Wd, _ = x.shape
    Ho, Wo = (H + stride - 1) // stride, (Wd + stride - 1) // stride
    xp = np.pad(x, ((0, 0), (pad, pad), (pad, pad), (0, 0)))
    z = np.zeros((B, Ho, Wo, W.shape[0]))
    for ky in range(k):
        for kx in range(k):
            patch = xp[:, ky:ky + stride * Ho:stride, kx:kx + stride * Wo:stride, :]
            z += patch @ W[:, ky * k + kx, :].T
    return z + b


def conv_backward(x, W, dz, stride, up):
    """Gradients of conv w.r.t. its input, weights and bias."""
    xin = x.repeat(2, axis=1).repeat(2, axis=2) if up else x
    taps = W.shape[1]
    k = 3 if taps == 9 else 1
    pad = k // 2
    B, H, Wd, _ = xin.shape
    Ho, Wo = dz.shape[1], dz.shape[2]
    xp = np.pad(xin, ((0, 0), (pad, pad), (pad, pad), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ky in range(k):
        for kx in range(k):
            sl = (slice(None), slice(ky, ky + stride * Ho, stride), slice(kx, kx + stride * Wo, stride))
            patch = xp[sl]
            dW[:, ky * k + kx, :] = np.einsum("byxo,byxi->oi", dz, patch)
            dxp[sl] += dz @ W[:, ky * k + kx, :]
    dx = dxp[:, pad:pad + H, pad:pad + Wd, :]
    if up:
        dx = dx.reshape(B, H // 2, 2, Wd // 2, 2, -1).sum(axis=(2, 4))
    db = dz.sum(axis=(0, 1, 2))
    return dx, dW, db


def forward(params, x, keep=False):
    """Returns the output (B, H, W, 3); with keep, also the per-layer cache."""
    acts = []          # layer outputs (post-activation)
    cache = []
    h = x
    for l, (ci, co, t, s, up, skip, act) in enumerate(ARCH):
        W, b = params[l]
        z = conv(h, W, b, s, up)
        if skip >= 0:
            z = z + acts[skip]
        a = z * sigmoid(z) if act else z
        cache.append((h, z))
        acts.append(a)
        h = a
    return (h, cache) if keep else h


def loss_and_grad(params, x, target, mask):
    """MSE over masked pixels and the 3 channels; returns (loss, grads list)."""
    out, cache = forward(params, x, keep=True)
    cnt = mask.sum() * out.shape[-1]
    diff = (out - target) * mask[..., None]
    loss = float((diff ** 2).sum() / cnt)
    dA = [None] * len(ARCH)
    dA[-1] = 2.0 * diff / cnt
    grads = [None] * len(ARCH)
    for l in range(len(ARCH) - 1, -1, -1):
        ci, co, t, s, up, skip, act = ARCH[l]
        h, z = cache[l]
        W, b = params[l]
        if act:
            sg = sigmoid(z)
            dz = dA[l] * sg * (1.0 + z * (1.0 - sg))
        else:
            dz = dA[l]
        dx, dW, db = conv_backward(h, W, dz, s, up)
        grads[l] = (dW, db)
        if skip >= 0:
            dA[skip] = dz if dA[skip] is None else dA[skip] + dz
        if l > 0:
            dA[l - 1] = dx if dA[l - 1] is None else dA[l - 1] + dx
    return loss, grads


def flatten(plist):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for (W, b) in plist])


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) with bias correction; t counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-style initialisation scaled by 1/sqrt(taps cin); zero biases."""
    rng = np.random.default_rng(seed)
    out = []
    for (ci, co, t, *_r) in ARCH:
        W = rng.standard_normal((co, t, ci)) * np.sqrt(2.0 / (t * ci))
        out.append((W, np.zeros(co)))
    return flatten(out)
