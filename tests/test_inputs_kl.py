"""Pins of the Gaussian-covariance expansion of eq. log_normal (problem data of
the paper's experiments) against facts independent of its separable Nystrom
construction: the eigenvalues of the full (non-separated) covariance matrix on
a midpoint grid, orthonormality and the eigen-equation checked by a 2D
Gauss-Legendre rule, the trace of the operator, Mercer's reconstruction of the
kernel, and the covariance of the generated log-coefficients."""
import numpy as np
import pytest

from paper_2302_13680_amd import inputs


def kernel(x1, y1, x2, y2, L2):
    return np.exp(-((x1 - x2) ** 2 + (y1 - y2) ** 2) / L2)


@pytest.mark.parametrize("L2", [0.5, 0.1])
def test_eigenvalues_match_the_full_covariance_matrix(L2):
    kl = inputs.gaussian_kl(8, L2)
    m = 40                                       # midpoint rule on a 40 x 40 grid
    t = (np.arange(m) + 0.5) / m
    X, Y = np.meshgrid(t, t)
    x, y = X.ravel(), Y.ravel()
    K = kernel(x[:, None], y[:, None], x[None], y[None], L2) / (m * m)
    ev = np.sort(np.linalg.eigvalsh(K))[::-1][:8]
    np.testing.assert_allclose(kl["lam"], ev, rtol=5e-3)


def test_trace_is_the_area():
    kl = inputs.gaussian_kl(4, 0.5, nq=60)
    assert abs(kl["mu"].sum() - 1.0) < 1e-12    # int_0^1 k(s, s) ds = 1, squared for 2D


@pytest.mark.parametrize("L2", [0.5, 0.1])
def test_modes_are_orthonormal_eigenfunctions(L2):
    kl = inputs.gaussian_kl(10, L2)
    s, w = np.polynomial.legendre.leggauss(50)
    s = 0.5 * (s + 1); w = 0.5 * w
    X, Y = np.meshgrid(s, s)
    W = np.outer(w, w)
    B = inputs.kl_modes(kl, X, Y)                # (10, 50, 50)
    G = np.einsum("aij,bij,ij->ab", B, B, W)
    np.testing.assert_allclose(G, np.eye(10), atol=1e-10)
    rng = np.random.default_rng(0)
    for _ in range(5):
        px, py = rng.uniform(0, 1, 2)
        Tb = np.einsum("ij,aij,ij->a", kernel(px, py, X, Y, L2), B, W)
        bp = inputs.kl_modes(kl, np.array(px), np.array(py))
        np.testing.assert_allclose(Tb, kl["lam"] * bp, rtol=1e-8, atol=1e-12)


def test_mercer_reconstruction_of_the_kernel():
    kl = inputs.gaussian_kl(60, 0.5)
    rng = np.random.default_rng(1)
    p = rng.uniform(0, 1, (20, 4))
    b1 = inputs.kl_modes(kl, p[:, 0], p[:, 1])
    b2 = inputs.kl_modes(kl, p[:, 2], p[:, 3])
    approx = np.einsum("m,mi,mi->i", kl["lam"], b1, b2)
    np.testing.assert_allclose(approx, kernel(p[:, 0], p[:, 1], p[:, 2], p[:, 3], 0.5), atol=1e-9)


def test_log_coefficients_have_the_covariance_of_the_field():
    """Monte Carlo covariance of log kappa at three faces, against
    sigma^2 sum_m lambda_m b_m(x) b_m(y) (M = 10 keeps 99.8% for L^2 = 0.5)."""
    sigma, L2, n, N = 0.7, 0.5, 7, 40000
    p = inputs.make_problem(n, N, 1e-4, M=10, sigma=sigma, seed=11, field="gaussian", corr_len2=L2)
    h = 1.0 / (n + 1)
    # kx[:, k, f] sits at ((f + 1/2) h, (k + 1) h)
    idx = [(0, 0), (3, 4), (6, 7)]
    pts = [((f + 0.5) * h, (k + 1) * h) for k, f in idx]
    g = np.stack([np.log(p.kx[:, k, f]) for k, f in idx])
    C = np.cov(g)
    kl = inputs.gaussian_kl(10, L2)
    for a in range(3):
        for b in range(3):
            ba = inputs.kl_modes(kl, np.array(pts[a][0]), np.array(pts[a][1]))
            bb = inputs.kl_modes(kl, np.array(pts[b][0]), np.array(pts[b][1]))
            exact = sigma ** 2 * np.sum(kl["lam"] * ba * bb)
            full = sigma ** 2 * kernel(*pts[a], *pts[b], L2)
            assert abs(C[a, b] - exact) <= 0.03 * sigma ** 2, (a, b, C[a, b], exact)
            assert abs(exact - full) <= 0.01 * sigma ** 2


def test_variance_kept_on_the_square():
    """The paper keeps M = 3 (L^2 = 0.5) and M = 15 (L^2 = 0.1) modes; on the unit
    square these keep 90.3% and 95.8% of the variance."""
    assert abs(inputs.gaussian_kl(3, 0.5)["variance_kept"] - 0.9033) < 1e-3
    assert abs(inputs.gaussian_kl(15, 0.1)["variance_kept"] - 0.9579) < 1e-3
