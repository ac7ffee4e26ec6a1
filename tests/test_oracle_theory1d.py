"""Pins of the oracle's node solve through the convergence theory of Section 3.1.

The collective Jacobi iteration matrix of the 1D model problem is built from
the oracle's node solve; its eigenvalues must be -mu_j lambda_i (Corollary
with Lemma spectrum_G) and the two-level operator must have the spectrum of
Theorem spectrum_two_level.
"""
import numpy as np
import pytest

from oracle import analysis1d as A


def _match(numeric, formula, tol):
    """every numeric eigenvalue lies within tol of some formula value, and the
    spectral radii agree"""
    numeric = np.asarray(numeric)
    formula = np.asarray(formula)
    for z in numeric:
        assert np.min(np.abs(formula - z)) <= tol, z
    assert abs(np.max(np.abs(numeric)) - np.max(np.abs(formula))) <= tol


@pytest.fixture(scope="module")
def model():
    Nh, N, nu = 15, 4, 1e-2
    eta = np.exp(np.random.default_rng(0).standard_normal(N) * 0.5)
    S, blocks = A.system_1d(Nh, eta, nu)
    Dinv = A.blockdiag_inverse_1d(Nh, blocks, N)
    return Nh, N, nu, eta, S, Dinv


def test_smoother_spectrum_lemma(model):
    Nh, N, nu, eta, S, Dinv = model
    G = A.jacobi_iteration_matrix(S, Dinv, 1.0)
    ev = np.linalg.eigvals(G)
    nz = ev[np.abs(ev) > 1e-6]
    formula = A.smoother_eigs(eta, nu, Nh)
    # 2N eigenvalues per frequency, the middle frequency contributes zeros
    assert len(nz) == 2 * N * Nh - 2 * N
    _match(nz, formula, 1e-6)
    rho = np.max(np.abs(ev))
    assert rho < 1.0


@pytest.mark.parametrize("n1,n2,theta", [(1, 1, 1.0), (2, 2, 1.0), (2, 2, 0.5), (1, 1, 0.8)])
def test_two_level_spectrum_theorem(model, n1, n2, theta):
    Nh, N, nu, eta, S, Dinv = model
    G = A.jacobi_iteration_matrix(S, Dinv, theta)
    T = A.two_level_operator(S, G, Nh, N, n1, n2)
    ev = np.linalg.eigvals(T)
    formula = A.theorem_spectrum_T(eta, nu, Nh, n1, n2, theta)
    nz = ev[np.abs(ev) > 1e-7]
    _match(nz, formula, 2e-6)
    assert np.max(np.abs(ev)) < 1.0


def test_nu_robustness_remark():
    """r -> 1 as nu -> 0, so |lambda_{2N-1,2N}| -> 0 (remark after the Lemma)."""
    eta = np.array([0.5, 1.0, 2.0])
    mags = []
    for nu in (1e-2, 1e-4, 1e-8):
        lam, r = A.lemma_spectrum_C(eta, nu, 15)
        mags.append(abs(lam[-1]))
    assert mags[0] > mags[1] > mags[2]
