"""Seeded synthetic problem instances for the linear-quadratic OCPUU.

This module only builds problem data: the random diffusion coefficients at
the cell faces, the block scalars and the right-hand side of the discrete
optimality system (Section 2, eq. full_space_optimality_system, rescaled to
its symmetric form).  It holds none of the multigrid method's arithmetic and
is shared by the GPU path and by the CPU oracle.

Discretization (5-point finite differences on the unit square, Dirichlet):
  * ``n`` interior nodes per direction, ``h = 1/(n+1)``; node ``(x, k)``
    (0-based) sits at ``((x+1) h, (k+1) h)``.
  * ``kx[j, k, f]`` (``f = 0..n``) is kappa_j at the x-face between nodes
    ``f-1`` and ``f`` of row ``k``, i.e. at ``((f+1/2) h, (k+1) h)``;
    ``ky[j, g, x]`` (``g = 0..n``) is kappa_j at ``((x+1) h, (g+1/2) h)``.
  * The stiffness matrix A_j is the h^2-scaled 5-point stencil built from
    those faces, the mass matrix is lumped, ``M = h^2 I``.

Blocks of S (eq. (2) notation): C_j = zeta_j h^2 I, G = nu h^2 I,
D_j = E_j = -h^2 I, with Monte Carlo weights zeta_j = 1/N or the weights of a
quadrature rule in the random variables (``stochastic_collocation``: tensor
Gauss-Hermite nodes and weights, the paper's SC setting).  Right-hand side:
f_Y,j = zeta_j h^2 y_d, f_U = 0, f_P,j = h^2 f.  This is the paper's system
with B = M after the adjoint is rescaled by zeta (the symmetrization remarked
on at the end of Section 2).

Coefficient model (Section 3.2, eq. log_normal, replaced by an analytic
Karhunen-Loeve-type expansion on the square):
  log kappa_j(x, y) = sum_{m=1..M} a_m xi_{j,m} sin(m pi x) sin(m pi y),
with xi drawn from ``numpy.random.default_rng(seed).standard_normal((N, M))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np


@dataclass
class Problem:
    n: int
    N: int
    nu: float
    kx: np.ndarray          # (N, n, n+1) float64
    ky: np.ndarray          # (N, n+1, n) float64
    c: np.ndarray           # (N,) C_j diagonal value
    d: np.ndarray           # (N,) D_j diagonal value
    e: np.ndarray           # (N,) E_j diagonal value
    g: float                # G diagonal value
    fY: np.ndarray          # (N, n, n)
    fU: np.ndarray          # (n, n)
    fP: np.ndarray          # (N, n, n)
    xi: np.ndarray = field(default=None, repr=False)
    yd: np.ndarray = field(default=None, repr=False)
    meta: dict = field(default_factory=dict)
    ctrl: np.ndarray = field(default=None, repr=False)   # (n, n) control mask, None: everywhere
    domain: np.ndarray = field(default=None, repr=False)  # (n, n) 1 inside / 0 outside, None: the square

    @property
    def h(self) -> float:
        return 1.0 / (self.n + 1)

    @property
    def dof(self) -> int:
        return (2 * self.N + 1) * self.n * self.n

    # --- layouts -----------------------------------------------------------
    # "paper" layout: x = [y_1..y_N | u | p_1..p_N], every block [n][n] (eq. (2)).
    # "node" layout (GPU): Y block [n][n][N], U block [n][n], P block [n][n][N]
    # (samples innermost), faces kx [n][n+1][N], ky [n+1][n][N].
    def rhs_paper(self) -> np.ndarray:
        return np.concatenate([self.fY.ravel(), self.fU.ravel(), self.fP.ravel()])

    def rhs_node(self) -> np.ndarray:
        return paper_to_node(self.rhs_paper(), self.n, self.N)

    def faces_node(self):
        return (np.ascontiguousarray(self.kx.transpose(1, 2, 0)),
                np.ascontiguousarray(self.ky.transpose(1, 2, 0)))


def paper_to_node(v: np.ndarray, n: int, N: int) -> np.ndarray:
    """Permute a vector from eq. (2) order to the node layout (samples innermost)."""
    nn = n * n
    v = np.asarray(v)
    Y = v[:N * nn].reshape(N, n, n).transpose(1, 2, 0)
    U = v[N * nn:(N + 1) * nn]
    P = v[(N + 1) * nn:].reshape(N, n, n).transpose(1, 2, 0)
    return np.concatenate([Y.ravel(), U.ravel(), P.ravel()])


def node_to_paper(v: np.ndarray, n: int, N: int) -> np.ndarray:
    nn = n * n
    v = np.asarray(v)
    Y = v[:N * nn].reshape(n, n, N).transpose(2, 0, 1)
    U = v[N * nn:(N + 1) * nn]
    P = v[(N + 1) * nn:].reshape(n, n, N).transpose(2, 0, 1)
    return np.concatenate([Y.ravel(), U.ravel(), P.ravel()])


def kl_amplitudes(M: int, sigma: float, decay: bool) -> np.ndarray:
    m = np.arange(1, M + 1, dtype=np.float64)
    return sigma / m if decay else np.full(M, sigma)


def log_kappa(xi: np.ndarray, amps: np.ndarray, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """log kappa_j at points (X, Y) for every sample j; returns (N,) + X.shape."""
    M = amps.shape[0]
    out = np.zeros((xi.shape[0],) + X.shape)
    for m in range(1, M + 1):
        mode = np.sin(m * math.pi * X) * np.sin(m * math.pi * Y)
        out += (amps[m - 1] * xi[:, m - 1])[:, None, None] * mode[None]
    return out


def gaussian_kl(M: int, corr_len2: float, nq: int = 80):
    """The M largest eigenpairs (lambda_m, b_m) of the covariance operator
    (T f)(x) = int_D exp(-|x - y|^2 / L^2) f(y) dy on the unit square D (eq.
    log_normal with unit variance: the paper's pairs are (b_m, sigma^2 lambda_m)).

    The kernel is a product of 1D kernels exp(-(s - t)^2 / L^2), so the 2D pairs
    are products mu_a mu_b, phi_a(x) phi_b(y) of the 1D ones, computed by the
    Nystrom method with nq Gauss-Legendre points on [0, 1] (the symmetric form
    W^1/2 K W^1/2) and evaluated anywhere by Nystrom interpolation.  Signs: every
    phi_a is positive at the first quadrature point; equal lambda are ordered by
    (a, b).  Returns a dict with lam (M,), the 1D index pairs, and what
    ``kl_modes`` needs."""
    s, w = np.polynomial.legendre.leggauss(nq)
    s = 0.5 * (s + 1.0)
    w = 0.5 * w
    K = np.exp(-(s[:, None] - s[None, :]) ** 2 / corr_len2)
    sw = np.sqrt(w)
    mu, V = np.linalg.eigh(sw[:, None] * K * sw[None, :])
    order = np.argsort(-mu, kind="stable")
    mu, V = mu[order], V[:, order]
    phi = V / sw[:, None]                       # phi_a at the quadrature points
    phi *= np.where(phi[0] < 0, -1.0, 1.0)[None, :]
    cand = sorted(((-(mu[a] * mu[b]), a, b) for a in range(min(nq, M + 1)) for b in range(min(nq, M + 1))))
    pairs = [(a, b) for _, a, b in cand[:M]]
    lam = np.array([mu[a] * mu[b] for a, b in pairs])
    return dict(lam=lam, pairs=pairs, mu=mu, s=s, w=w, phi=phi, corr_len2=float(corr_len2),
                variance_kept=float(lam.sum()))


def kl_modes(kl, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """b_m(X, Y) for every mode of ``gaussian_kl``: shape (M,) + X.shape."""
    s, w, phi, mu, L2 = kl["s"], kl["w"], kl["phi"], kl["mu"], kl["corr_len2"]

    def phi_at(a, t):   # Nystrom interpolation of the 1D eigenfunction a
        t = np.asarray(t, dtype=np.float64)
        k = np.exp(-(t[..., None] - s) ** 2 / L2)
        return (k @ (w * phi[:, a])) / mu[a]
    return np.stack([phi_at(a, X) * phi_at(b, Y) for a, b in kl["pairs"]])


def stochastic_collocation(M: int, q: int):
    """Tensor Gauss-Hermite rule for M independent standard normal variables with
    q points per variable: nodes xi (q^M, M) and weights zeta (q^M,) summing to 1
    (Section 3.2's stochastic collocation; numpy's probabilists' Hermite rule,
    weight exp(-t^2/2), normalized).  Node j has digits (i_1..i_M) in base q, the
    last variable fastest."""
    t, w = np.polynomial.hermite_e.hermegauss(q)
    w = w / w.sum()
    idx = np.array(np.meshgrid(*([np.arange(q)] * M), indexing="ij")).reshape(M, -1).T
    xi = t[idx]
    zeta = np.prod(w[idx], axis=1)
    return xi, zeta


def make_problem(n: int, N: int, nu: float = 1e-4, *, M: int = 4, sigma: float = 0.5,
                 decay: bool = False, seed: int = 0, yd: str | np.ndarray = "sin",
                 f: float = 1.0, xi: np.ndarray | None = None,
                 kappa_const: float | None = None, weights: np.ndarray | None = None,
                 control_region: tuple | None = None, field: str = "sine",
                 corr_len2: float = 0.5, domain: str = "square", rows: str = "scaled") -> Problem:
    """Build one seeded instance.

    ``decay=False`` gives amplitudes a_m = sigma (the 31x31, N=8 case, four modes
    of amplitude 0.5); ``decay=True`` gives a_m = sigma/m.  ``kappa_const`` replaces
    the random field by a constant (used by closed-form checks).  ``field =
    "gaussian"`` takes the paper's expansion instead (eq. log_normal):
    log kappa_j = sigma sum_m sqrt(lambda_m) b_m xi_{j,m} with the eigenpairs of
    the Gaussian covariance of correlation length^2 ``corr_len2`` on the unit
    square (``gaussian_kl``); sigma is then the field's standard deviation.
    ``domain = "lshape"``: the paper's L-shaped domain (0,1)^2 minus [1/2,1)^2,
    as the nodes of the square grid with x < 1/2 or y < 1/2 (nodes outside are
    homogeneous Dirichlet nodes; the right-hand side is zero there).  ``weights`` are
    the quadrature weights zeta_j of the samples (default 1/N, Monte Carlo).
    ``control_region = (x0, x1, y0, y1)`` restricts the control to the nodes in
    the closed rectangle [x0, x1] x [y0, y1] (local control; the mask of the
    node entries of D_j and E_j); None lets it act everywhere.
    ``rows``: "scaled" (default) carries the adjoint rescaled by the weights
    (p~_j = zeta_j p_j, Y rows times zeta_j: C_j = zeta_j h^2, D_j = -h^2, the
    symmetric form); "paper" keeps the rows as printed in eq.
    full_space_optimality_system (C_j = M = h^2 I, D_j = -zeta_j h^2 I,
    f_Y,j = h^2 y_d).  The two give the same iterates of the collective smoother
    and of the multigrid hierarchy (a node-block scaling), but a residual norm,
    and so a stopping test or a GMRES minimization, weighted differently.
    """
    h = 1.0 / (n + 1)
    if xi is None:
        xi = np.random.default_rng(seed).standard_normal((N, M))
    xi = np.asarray(xi, dtype=np.float64)
    amps = kl_amplitudes(xi.shape[1], sigma, decay)
    nodes = (np.arange(n) + 1.0) * h
    faces = (np.arange(n + 1) + 0.5) * h
    if kappa_const is not None:
        kx = np.full((N, n, n + 1), float(kappa_const))
        ky = np.full((N, n + 1, n), float(kappa_const))
    elif field == "gaussian":
        kl = gaussian_kl(xi.shape[1], corr_len2)
        coef = sigma * np.sqrt(kl["lam"])[None, :] * xi          # (N, M)
        FX, KY_ = np.meshgrid(faces, nodes)
        kx = np.exp(np.tensordot(coef, kl_modes(kl, FX, KY_), axes=1))
        XN, GF = np.meshgrid(nodes, faces)
        ky = np.exp(np.tensordot(coef, kl_modes(kl, XN, GF), axes=1))
    elif field != "sine":
        raise ValueError(field)
    else:
        FX, KY_ = np.meshgrid(faces, nodes)          # kx: rows k (y = nodes), faces f (x = faces)
        kx = np.exp(log_kappa(xi, amps, FX, KY_))
        XN, GF = np.meshgrid(nodes, faces)           # ky: rows g (y = faces), columns x (x = nodes)
        ky = np.exp(log_kappa(xi, amps, XN, GF))
    XX, YY = np.meshgrid(nodes, nodes)
    if isinstance(yd, str):
        if yd == "sin":
            ydv = np.sin(math.pi * XX) * np.sin(math.pi * YY)
        elif yd == "zero":
            ydv = np.zeros((n, n))
        else:
            raise ValueError(yd)
    else:
        ydv = np.asarray(yd, dtype=np.float64).reshape(n, n)
    zeta = np.full(N, 1.0 / N) if weights is None else np.asarray(weights, dtype=np.float64)
    if zeta.shape != (N,) or not np.all(zeta > 0):
        raise ValueError("weights must be N positive numbers")
    if rows == "scaled":
        c = zeta * h * h
        d = np.full(N, -h * h)
        fY = (zeta * h * h)[:, None, None] * ydv[None]
    elif rows == "paper":
        c = np.full(N, h * h)
        d = -zeta * h * h
        fY = np.repeat((h * h * ydv)[None], N, axis=0)
    else:
        raise ValueError(rows)
    e = np.full(N, -h * h)
    g = nu * h * h
    fU = np.zeros((n, n))
    fP = np.full((N, n, n), h * h * f)
    dom = None
    if domain == "lshape":
        eps = 1e-12
        dom = (~((XX >= 0.5 - eps) & (YY >= 0.5 - eps))).astype(np.float64)
        fY = fY * dom[None]
        fP = fP * dom[None]
    elif domain != "square":
        raise ValueError(domain)
    ctrl = None
    if control_region is not None:
        x0, x1, y0, y1 = control_region
        eps = 1e-12
        ctrl = (((XX >= x0 - eps) & (XX <= x1 + eps) & (YY >= y0 - eps) & (YY <= y1 + eps))
                .astype(np.float64))
    return Problem(n=n, N=N, nu=nu, kx=np.ascontiguousarray(kx), ky=np.ascontiguousarray(ky),
                   c=c, d=d, e=e, g=g, fY=fY, fU=fU, fP=fP, xi=xi, yd=ydv, ctrl=ctrl, domain=dom,
                   meta=dict(M=xi.shape[1], sigma=sigma, decay=decay, seed=seed, f=f, field=field,
                             quadrature="mc" if weights is None else "weights"))


def collocation_problem(n: int, q: int, nu: float = 1e-4, *, M: int = 3, sigma: float = 0.5,
                        decay: bool = True, **kw) -> Problem:
    """The same model with the N = q^M tensor Gauss-Hermite nodes as samples and
    their weights as zeta_j (the paper's SC columns use M = 3, N in {8, 27, 64, 125})."""
    xi, zeta = stochastic_collocation(M, q)
    return make_problem(n, xi.shape[0], nu, M=M, sigma=sigma, decay=decay, xi=xi, weights=zeta, **kw)


def paper_target(n: int) -> np.ndarray:
    """y_d = exp(y^2) sin(2 pi x) sin(2 pi y) at the interior nodes, the target
    state of the paper's experiments (Section 3.2 and after)."""
    t = (np.arange(n) + 1.0) / (n + 1)
    X, Y = np.meshgrid(t, t)
    return np.exp(Y ** 2) * np.sin(2 * math.pi * X) * np.sin(2 * math.pi * Y)


def boundary_control_problem(n: int, N: int, nu: float = 1e-4, *, M: int = 3, sigma: float = 0.5,
                             decay: bool = True, seed: int = 0, field: str = "sine", corr_len2: float = 0.5,
                             weights: np.ndarray | None = None, xi: np.ndarray | None = None,
                             f: float = 0.0, rows: str = "scaled") -> Problem:
    """Neumann boundary control on Gamma = (0,1) x {0} of the unit square (the
    paper's boundary-control table), Dirichlet on the rest of the boundary.

    Built by reflection: the state and adjoint extend evenly across Gamma to the
    rectangle (0,1) x (-1,1), where the boundary control becomes a control on the
    mirror line.  That rectangle is the left half (the domain; the right half is
    removed) of an n x n grid of the square (0,1)^2 scaled by 2, so the physical
    spacing is h = 2/(n+1): 15x16, 31x32 and 63x64 physical nodes (the paper's
    N_h = 240, 992, 4032) for n = 31, 63, 127; the mirror row is a grid line of
    every level.  Restricted to y >= 0 the even system is the half-cell
    discretization of the Neumann row (half faces along Gamma, half mass, boundary
    flux h u).  Blocks: C_j = zeta_j h^2 I, D_j = E_j = -2 h (the line source of
    both halves), G = 2 nu h (the doubled cost), the control acting on the mirror
    row only; on coarse levels D_j, E_j and G grow x2 per coarsening (the 1D mass
    of a line, meta["control_growth"]) while C_j grows x4; kappa, y_d (the paper's target) and f taken at (x, |y|).  The
    coefficient models are those of ``make_problem`` evaluated at physical
    points; the solution's U block on the mirror row is the boundary control, its
    Y and P blocks above it (and on it) the state and the adjoint.  ``rows`` as
    in ``make_problem`` ("paper": C_j = h^2 I, D_j = -2 zeta_j h I, f_Y = h^2 y_d)."""
    if n < 3 or (n + 1) % 4:
        raise ValueError("n + 1 must be a multiple of 4")
    H = 2.0 / (n + 1)                                   # physical spacing
    if xi is None:
        xi = np.random.default_rng(seed).standard_normal((N, M))
    xi = np.asarray(xi, dtype=np.float64)
    zeta = np.full(N, 1.0 / N) if weights is None else np.asarray(weights, dtype=np.float64)
    g_nodes = (np.arange(n) + 1.0) / (n + 1)            # grid coordinates in (0, 1)
    g_faces = (np.arange(n + 1) + 0.5) / (n + 1)
    px = lambda X: 2.0 * X                              # physical x
    py = lambda Y: np.abs(2.0 * Y - 1.0)                # physical |y|

    def log_field(X, Y):
        if field == "gaussian":
            kl = gaussian_kl(xi.shape[1], corr_len2)
            coef = sigma * np.sqrt(kl["lam"])[None, :] * xi
            return np.tensordot(coef, kl_modes(kl, px(X), py(Y)), axes=1)
        if field != "sine":
            raise ValueError(field)
        return log_kappa(xi, kl_amplitudes(xi.shape[1], sigma, decay), px(X), py(Y))

    FX, KY_ = np.meshgrid(g_faces, g_nodes)
    kx = np.exp(log_field(FX, KY_))
    XN, GF = np.meshgrid(g_nodes, g_faces)
    ky = np.exp(log_field(XN, GF))
    XX, YY = np.meshgrid(g_nodes, g_nodes)
    xp, yp = px(XX), py(YY)
    ydv = np.exp(yp ** 2) * np.sin(2 * math.pi * xp) * np.sin(2 * math.pi * yp)
    mid = (n + 1) // 2 - 1                              # the mirror row (y = 0)
    dom = (XX < 0.5 - 1e-12).astype(np.float64)         # x < 1
    ctrl = np.zeros((n, n))
    ctrl[mid, :] = dom[mid, :]
    if rows == "scaled":
        c = zeta * H * H
        d = np.full(N, -2.0 * H)
        fY = (zeta * H * H)[:, None, None] * (ydv * dom)[None]
    elif rows == "paper":
        c = np.full(N, H * H)
        d = -2.0 * H * zeta
        fY = np.repeat((H * H * ydv * dom)[None], N, axis=0)
    else:
        raise ValueError(rows)
    e = np.full(N, -2.0 * H)
    g = 2.0 * nu * H
    fU = np.zeros((n, n))
    fP = np.full((N, n, n), H * H * f) * dom[None]
    return Problem(n=n, N=N, nu=nu, kx=np.ascontiguousarray(kx), ky=np.ascontiguousarray(ky), c=c, d=d, e=e, g=g,
                   fY=fY, fU=fU, fP=fP, xi=xi, yd=ydv, ctrl=ctrl, domain=dom,
                   meta=dict(M=xi.shape[1], sigma=sigma, decay=decay, seed=seed, f=f, field=field,
                             boundary_control=True, h=H, mirror_row=mid, control_growth=2.0,
                             quadrature="mc" if weights is None else "weights"))


def boundary_collocation_problem(n: int, q: int, nu: float = 1e-4, *, M: int = 3, **kw) -> Problem:
    """``boundary_control_problem`` with q^M tensor Gauss-Hermite nodes and weights."""
    xi, zeta = stochastic_collocation(M, q)
    return boundary_control_problem(n, xi.shape[0], nu, M=M, xi=xi, weights=zeta, **kw)


def random_yd(n: int, rng: np.random.Generator, terms: int = 3, kmax: int = 4) -> np.ndarray:
    """Target state drawn as a random sum of ``terms`` sine products
    sum_t c_t sin(k_t pi x) sin(l_t pi y), c_t ~ U[-1, 1], k_t, l_t ~ U{1..kmax}."""
    h = 1.0 / (n + 1)
    nodes = (np.arange(n) + 1.0) * h
    XX, YY = np.meshgrid(nodes, nodes)
    out = np.zeros((n, n))
    for _ in range(terms):
        ct = rng.uniform(-1.0, 1.0)
        kk = int(rng.integers(1, kmax + 1))
        ll = int(rng.integers(1, kmax + 1))
        out += ct * np.sin(kk * math.pi * XX) * np.sin(ll * math.pi * YY)
    return out


# Named workloads of the evaluation (sizes from the experiment plan).
def small_fp64(seed: int = 0) -> Problem:
    """31x31 interior grid, N=8, four modes of amplitude 0.5, nu=1e-4."""
    return make_problem(31, 8, 1e-4, M=4, sigma=0.5, decay=False, seed=seed)


def medium_fp64(seed: int = 1) -> Problem:
    """255x255 interior grid, N=64, six modes of amplitude 0.5/m, nu=1e-4."""
    return make_problem(255, 64, 1e-4, M=6, sigma=0.5, decay=True, seed=seed)


def large_mixed(seed: int = 2) -> Problem:
    """511x511 interior grid, N=256, six modes of amplitude 1.0/m, nu=1e-4."""
    return make_problem(511, 256, 1e-4, M=6, sigma=1.0, decay=True, seed=seed)


def batch_instances(count: int = 64, draw_seed: int = 999, first_seed: int = 1000):
    """Uneven batch: n ~ U{63,127,255}, N ~ U{16,32,64,128}, log10 nu ~ U[-6,-2]."""
    rng = np.random.default_rng(draw_seed)
    out = []
    for i in range(count):
        n = int(rng.choice([63, 127, 255]))
        N = int(rng.choice([16, 32, 64, 128]))
        nu = float(10.0 ** rng.uniform(-6.0, -2.0))
        out.append(dict(n=n, N=N, nu=nu, seed=first_seed + i))
    return out


def learned_instance(seed: int, n: int = 127, N: int = 128) -> Problem:
    """Warm-start workload: nu log-uniform in [1e-5, 1e-3], y_d a random sum of
    three sine products, f = 1, six modes of amplitude 0.5/m."""
    nu, yd, xi = learned_instance_params(seed, n, N)
    return make_problem(n, N, nu, M=6, sigma=0.5, decay=True, seed=seed, yd=yd, xi=xi)


def make_problem_device(n: int, N: int, nu: float, xi, yd, *, sigma: float = 0.5, decay: bool = True,
                        f: float = 1.0, device="cuda"):
    """The same instance as ``make_problem`` (analytic KL coefficients at the
    faces, Monte Carlo weights, f = 1), generated directly on the device in the
    node layout.  Returns (kx, ky, rhs, c, d, e, g): torch FP64 device tensors
    for the faces and right-hand side, numpy arrays / float for the blocks."""
    import torch
    h = 1.0 / (n + 1)
    xi = torch.as_tensor(np.asarray(xi, dtype=np.float64), device=device)
    M = xi.shape[1]
    amps = torch.as_tensor(kl_amplitudes(M, sigma, decay), device=device)
    nodes = (torch.arange(n, device=device, dtype=torch.float64) + 1.0) * h
    faces = (torch.arange(n + 1, device=device, dtype=torch.float64) + 0.5) * h
    m = torch.arange(1, M + 1, device=device, dtype=torch.float64)
    sn = torch.sin(math.pi * m[:, None] * nodes[None, :])       # (M, n)
    sf = torch.sin(math.pi * m[:, None] * faces[None, :])       # (M, n+1)
    w = amps[None, :] * xi                                      # (N, M)
    # kx[k][f][j] = exp(sum_m w[j, m] sin(m pi f_x) sin(m pi y_k)); ky[g][x][j] likewise
    kx = torch.exp(torch.einsum("jm,mk,mf->kfj", w, sn, sf)).contiguous()
    ky = torch.exp(torch.einsum("jm,mg,mx->gxj", w, sf, sn)).contiguous()
    ydv = torch.as_tensor(np.asarray(yd, dtype=np.float64), device=device).reshape(n, n)
    zeta = 1.0 / N
    c = np.full(N, zeta * h * h)
    d = np.full(N, -h * h)
    e = np.full(N, -h * h)
    g = nu * h * h
    fY = (zeta * h * h) * ydv[:, :, None].expand(n, n, N)
    fP = torch.full((n, n, N), h * h * f, dtype=torch.float64, device=device)
    fU = torch.zeros(n * n, dtype=torch.float64, device=device)
    rhs = torch.cat([fY.reshape(-1), fU, fP.reshape(-1)]).contiguous()
    return kx, ky, rhs, c, d, e, g


def learned_instance_params(seed: int, n: int = 127, N: int = 128):
    """Random draws of the warm-start workload for one seed: (nu, y_d, xi)."""
    rng = np.random.default_rng(seed)
    nu = float(10.0 ** rng.uniform(-5.0, -3.0))
    yd = random_yd(n, rng)
    xi = rng.standard_normal((N, 6))
    return nu, yd, xi
