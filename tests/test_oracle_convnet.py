"""Pins of the FP64 reference network: gradients against central finite
differences, the convolution against a direct loop, the bf16 rounding rule,
and Adam against its closed form on a quadratic."""
import numpy as np
import pytest

from oracle import convnet as cn


def test_param_count_is_about_150k():
    assert 140_000 <= cn.n_params() <= 180_000


def test_conv_matches_direct_loops():
    rng = np.random.default_rng(0)
    for (stride, up, taps) in [(1, 0, 9), (2, 0, 9), (1, 1, 9), (1, 0, 1)]:
        H = 6 if not up else 3
        x = rng.standard_normal((2, H, H, 3))
        W = rng.standard_normal((4, taps, 3))
        b = rng.standard_normal(4)
        z = cn.conv(x, W, b, stride, up)
        xi = x.repeat(2, 1).repeat(2, 2) if up else x
        Hi = xi.shape[1]
        k = 3 if taps == 9 else 1
        Ho = (Hi + stride - 1) // stride
        ref = np.zeros((2, Ho, Ho, 4))
        for bb in range(2):
            for yo in range(Ho):
                for xo in range(Ho):
                    for co in range(4):
                        s = b[co]
                        for ky in range(k):
                            for kx in range(k):
                                yy = stride * yo + ky - k // 2
                                xx = stride * xo + kx - k // 2
                                if 0 <= yy < Hi and 0 <= xx < Hi:
                                    s += W[co, ky * k + kx] @ xi[bb, yy, xx]
                        ref[bb, yo, xo, co] = s
        np.testing.assert_allclose(z, ref, rtol=1e-12, atol=1e-12)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    theta = cn.init_params(seed=2) + 0.01 * rng.standard_normal(cn.n_params())
    params = cn.unflatten(theta)
    H = 16
    x = rng.standard_normal((2, H, H, 4))
    t = rng.standard_normal((2, H, H, 3))
    mask = np.ones((2, H, H))
    mask[:, -1, :] = 0
    mask[:, :, -1] = 0
    loss, grads = cn.loss_and_grad(params, x, t, mask)
    g = cn.flatten(grads)
    idx = rng.choice(cn.n_params(), 40, replace=False)
    eps = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += eps
        tm = theta.copy(); tm[i] -= eps
        lp, _ = cn.loss_and_grad(cn.unflatten(tp), x, t, mask)
        lm, _ = cn.loss_and_grad(cn.unflatten(tm), x, t, mask)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_input_gradient_matches_central_differences():
    """The chain through skips and upsampling also reaches the input."""
    rng = np.random.default_rng(3)
    params = cn.unflatten(cn.init_params(seed=4))
    H = 8
    x = rng.standard_normal((1, H, H, 4))
    t = rng.standard_normal((1, H, H, 3))
    mask = np.ones((1, H, H))

    def loss_of(xx):
        out = cn.forward(params, xx)
        return ((out - t) ** 2).sum() / (mask.sum() * 3)

    # analytic input gradient: run the backward with an extra identity layer is not
    # available, so compare d loss / d x through the first layer's conv_backward
    out, cache = cn.forward(params, x, keep=True)
    _, grads = cn.loss_and_grad(params, x, t, mask)
    # finite differences on a few input entries, checked against the weights'
    # linearity: perturbing x changes the loss consistently with the first layer
    for _ in range(5):
        i = tuple(rng.integers(0, s) for s in x.shape)
        e = 1e-6
        xp = x.copy(); xp[i] += e
        xm = x.copy(); xm[i] -= e
        fd = (loss_of(xp) - loss_of(xm)) / (2 * e)
        # analytic: recompute with the backward chain down to the input
        dA = 2.0 * (out - t) / (mask.sum() * 3)
        h = dA
        dAs = [None] * len(cn.ARCH)
        dAs[-1] = dA
        dx0 = None
        for l in range(len(cn.ARCH) - 1, -1, -1):
            ci, co, tp, s, up, skip, act = cn.ARCH[l]
            hin, z = cache[l]
            W, b = params[l]
            sg = cn.sigmoid(z)
            dz = dAs[l] * sg * (1 + z * (1 - sg)) if act else dAs[l]
            dx, _, _ = cn.conv_backward(hin, W, dz, s, up)
            if skip >= 0:
                dAs[skip] = dz if dAs[skip] is None else dAs[skip] + dz
            if l > 0:
                dAs[l - 1] = dx if dAs[l - 1] is None else dAs[l - 1] + dx
            else:
                dx0 = dx
        assert abs(fd - dx0[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9


def test_bf16_round_to_nearest_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert cn.bf16_round(1.0 + 2.0 ** -8) == 1.0
    assert cn.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert cn.bf16_round(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7
    v = np.random.default_rng(0).standard_normal(1000)
    r = cn.bf16_round(v)
    assert np.all(np.abs(r - v) <= np.abs(v) * 2.0 ** -8 + 1e-30)


def test_adam_closed_form_first_step():
    """With bias correction the first Adam step moves every coordinate by lr sign(g)
    (up to eps)."""
    theta = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    new, m, v = cn.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(new, theta - 0.01 * np.sign(g), rtol=0, atol=1e-7)
