"""1D model problem of the convergence analysis (Section 3.1).

TEST INFRASTRUCTURE ONLY.  Builds the finite-difference optimality system of
eq. full_space_optimality_system_simplified (N Monte Carlo samples of a
scaled 1D Laplacian, symmetric form), the collective Jacobi iteration matrix
of eq. collective_smoothing (node blocks inverted by the oracle's node solve,
eq. solution_reduced_system), the two-level operator with a Galerkin coarse
matrix, full weighting and linear interpolation, and the closed forms of
Lemma spectrum_G (spectrum of C), Corollary (eigenvalues -mu_j lambda_i of the
smoother) and Theorem spectrum_two_level (spectrum of T).
"""
from __future__ import annotations

import numpy as np

from .oracle import node_solve


def system_1d(Nh: int, eta: np.ndarray, nu: float):
    """Dense S of eq. full_space_optimality_system_simplified, unknowns ordered
    (y_1..y_N, u, p_1..p_N), each block of length Nh.  Returns S and the node
    block data (a, c, d, e, g) used by the node solve."""
    N = len(eta)
    h = 1.0 / (Nh + 1)
    A = (2.0 * np.eye(Nh) - np.eye(Nh, k=1) - np.eye(Nh, k=-1)) / h ** 2
    I = np.eye(Nh)
    n = (2 * N + 1) * Nh
    S = np.zeros((n, n))
    Y = lambda j: slice(j * Nh, (j + 1) * Nh)
    U = slice(N * Nh, (N + 1) * Nh)
    P = lambda j: slice((N + 1 + j) * Nh, (N + 2 + j) * Nh)
    for j in range(N):
        S[Y(j), Y(j)] = I / N
        S[Y(j), P(j)] = eta[j] / N * A
        S[P(j), Y(j)] = eta[j] / N * A
        S[P(j), U] = -I / N
        S[U, P(j)] = -I / N
    S[U, U] = nu * I
    blocks = dict(a=eta / N * 2.0 / h ** 2, c=np.full(N, 1.0 / N), d=np.full(N, -1.0 / N),
                  e=np.full(N, -1.0 / N), g=nu)
    return S, blocks


def node_index(Nh: int, N: int, i: int):
    """Indices R_i of eq. restriction_action in the (y, u, p) ordering, returned
    in the order (y~_i, u_i, p~_i) expected by the node solve's block rows."""
    ys = [j * Nh + i for j in range(N)]
    us = [N * Nh + i]
    ps = [(N + 1 + j) * Nh + i for j in range(N)]
    return ys, us, ps


def blockdiag_inverse_1d(Nh: int, blocks: dict, N: int) -> np.ndarray:
    """sum_i P_i S~_i^{-1} R_i with every S~_i^{-1} applied through the oracle's
    node solve (probed on unit right-hand sides)."""
    n = (2 * N + 1) * Nh
    Dinv = np.zeros((n, n))
    a, c, d, e, g = blocks["a"], blocks["c"], blocks["d"], blocks["e"], blocks["g"]
    for i in range(Nh):
        ys, us, ps = node_index(Nh, N, i)
        idx = ys + us + ps
        for q in range(2 * N + 1):
            b = np.zeros(2 * N + 1)
            b[q] = 1.0
            # block rows of eq. reduced_matrices: first row (C, A) <- y~ rows of S,
            # second row (G, D) <- u row, third row (A, E) <- p~ rows.
            bP, bU, bY = b[:N], b[N], b[N + 1:]
            y, u, p = node_solve(a, c, d, e, g, bP, bU, bY)
            Dinv[np.ix_(ys, [idx[q]])] = y[:, None]
            Dinv[us[0], idx[q]] = u
            Dinv[np.ix_(ps, [idx[q]])] = p[:, None]
    return Dinv


def jacobi_iteration_matrix(S, Dinv, theta: float = 1.0):
    n = S.shape[0]
    return np.eye(n) - theta * Dinv @ S


def interpolation_1d(Nh: int) -> np.ndarray:
    """Linear interpolation from Nh_c = (Nh-1)/2 coarse to Nh fine nodes."""
    Nc = (Nh - 1) // 2
    P = np.zeros((Nh, Nc))
    for I in range(Nc):
        P[2 * I + 1, I] = 1.0
        P[2 * I, I] = 0.5
        P[2 * I + 2, I] = 0.5
    return P


def two_level_operator(S, G, Nh: int, N: int, n1: int, n2: int):
    """T = G^{n2} (I - P (R S P)^{-1} R S) G^{n1}, with R = P^T and P the linear
    interpolation applied to every one of the 2N+1 fields (R = R~ (x) I)."""
    Pt = interpolation_1d(Nh)
    P = np.kron(np.eye(2 * N + 1), Pt)
    R = P.T
    Sc = R @ S @ P
    K = np.eye(S.shape[0]) - P @ np.linalg.solve(Sc, R @ S)
    return np.linalg.matrix_power(G, n2) @ K @ np.linalg.matrix_power(G, n1)


# ------------------------------------------------------------ closed forms
def lemma_spectrum_C(eta: np.ndarray, nu: float, Nh: int):
    """Lemma spectrum_G: sigma(C) = -1/2 {1 (x 2N-2), 1 - r +- i sqrt((1-r) r)},
    r = E^[d~^-2] / (nu + E^[d~^-2]), d~_j = N d_j = 2 eta_j / h^2."""
    N = len(eta)
    h = 1.0 / (Nh + 1)
    dt = 2.0 * eta / h ** 2
    Ed = np.mean(dt ** -2.0)
    r = Ed / (nu + Ed)
    lam = [-0.5] * (2 * N - 2)
    z = (1 - r) + 1j * np.sqrt((1 - r) * r)
    lam += [-0.5 * z, -0.5 * np.conj(z)]
    return np.array(lam, dtype=complex), r


def smoother_eigs(eta, nu, Nh):
    """Corollary: delta_{i,j} = -mu_j lambda_i, mu_j = 2 cos(j pi/(Nh+1))."""
    lam, _ = lemma_spectrum_C(eta, nu, Nh)
    mu = 2 * np.cos(np.arange(1, Nh + 1) * np.pi / (Nh + 1))
    return np.array([-m * l for m in mu for l in lam])


def theorem_spectrum_T(eta, nu, Nh, n1, n2, theta: float = 1.0):
    """Theorem spectrum_two_level (n = n1 + n2 smoothing steps), with the
    damped factor 1 - theta + theta delta in place of delta (damping remark)."""
    lam, _ = lemma_spectrum_C(eta, nu, Nh)
    nn = n1 + n2
    out = []
    h = 1.0 / (Nh + 1)
    for j in range(1, (Nh + 1) // 2):
        jt = Nh + 1 - j
        cj2 = np.cos(j * np.pi * h / 2) ** 2
        sj2 = np.sin(j * np.pi * h / 2) ** 2
        muj = 2 * np.cos(j * np.pi * h)
        mujt = 2 * np.cos(jt * np.pi * h)
        for li in lam:
            dj = -muj * li
            djt = -mujt * li
            gj = 1 - theta + theta * dj
            gjt = 1 - theta + theta * djt
            # the coarse-correction weights use the undamped S-block factors 1 - delta
            num = cj2 ** 2 * (1 - dj) * gjt ** nn + sj2 ** 2 * (1 - djt) * gj ** nn
            den = cj2 ** 2 * (1 - dj) + sj2 ** 2 * (1 - djt)
            out.append(num / den)
    # frequency jbar = (Nh+1)/2: mu = 0, the restriction annihilates it and the
    # damped smoother leaves the factor (1 - theta) per step
    out.extend([(1 - theta) ** nn] * len(lam))
    return np.array(out)
