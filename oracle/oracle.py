"""ctypes wrapper of the C oracle (``smg_oracle.c``) plus small helpers.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Vectors use the
paper's layout of eq. (2): x = [y_1..y_N | u | p_1..p_N], each block n x n.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smg_oracle.c")
_LIB = os.path.join(_HERE, "libsmg_oracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def oracle_lib_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, OpenMP over independent nodes)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-Wno-unused-function", "-Wno-maybe-uninitialized", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build_oracle()
    L = C.CDLL(_LIB)
    vp = C.c_void_p
    L.or_set_smoother.argtypes = [vp, C.c_int]
    L.or_set_control.restype = C.c_int
    L.or_set_control.argtypes = [vp, _dp]
    L.or_set_sample_c.restype = C.c_int
    L.or_set_sample_c.argtypes = [vp, _dp]
    L.or_set_control_growth.restype = C.c_int
    L.or_set_control_growth.argtypes = [vp, C.c_double]
    L.or_set_domain.restype = C.c_int
    L.or_set_domain.argtypes = [vp, _dp]
    L.or_set_masks.restype = C.c_int
    L.or_set_masks.argtypes = [vp, C.c_void_p, C.c_void_p, C.c_int]
    L.or_level_factor.argtypes = [vp, C.c_int, C.c_int, _dp]
    L.or_level_domain.argtypes = [vp, C.c_int, _dp]
    L.or_create.restype = vp
    L.or_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                            _dp, _dp, _dp, _dp, _dp, C.c_double]
    L.or_destroy.argtypes = [vp]
    L.or_nlevels.argtypes = [vp]
    L.or_level_n.argtypes = [vp, C.c_int]
    L.or_level_faces.argtypes = [vp, C.c_int, _dp, _dp]
    L.or_level_scalars.argtypes = [vp, C.c_int, _dp, _dp, _dp, C.POINTER(C.c_double)]
    L.or_apply.argtypes = [vp, C.c_int, _dp, _dp]
    L.or_residual.argtypes = [vp, C.c_int, _dp, _dp, _dp]
    L.or_halfsweep.argtypes = [vp, C.c_int, C.c_int, C.c_double, _dp, _dp]
    L.or_halfsweep32.argtypes = [vp, C.c_int, C.c_int, C.c_double, _dp, _dp]
    L.or_jacobi.argtypes = [vp, C.c_int, C.c_double, _dp, _dp]
    L.or_restrict.argtypes = [C.c_int, C.c_int, _dp, _dp]
    L.or_residual_restrict.argtypes = [vp, C.c_int, _dp, _dp, _dp]
    L.or_prolong_control.argtypes = [vp, C.c_int, _dp, _dp]
    L.or_prolong_add.argtypes = [C.c_int, C.c_int, _dp, _dp]
    L.or_coarsen_faces.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp]
    L.or_coarse_solve.argtypes = [vp, _dp, _dp]
    L.or_node_solve.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_double, _dp, C.c_double, _dp,
                                _dp, C.POINTER(C.c_double), _dp]
    L.or_vcycle.argtypes = [vp, _dp, _dp, C.c_int]
    L.or_vcycle32.argtypes = [vp, _dp, _dp, C.c_int]
    L.or_solve_vcycle.restype = C.c_int
    L.or_solve_vcycle.argtypes = [vp, _dp, _dp, C.c_double, C.c_int, _dp]
    L.or_gmres.restype = C.c_int
    L.or_gmres.argtypes = [vp, _dp, _dp, C.c_int, C.c_double, C.c_int, C.c_int, _dp]
    L.or_solve_ir.restype = C.c_int
    L.or_solve_ir.argtypes = [vp, _dp, _dp, C.c_double, C.c_double, C.c_int, C.c_int, _dp,
                              C.POINTER(C.c_int)]
    L.or_num_threads.restype = C.c_int
    L.or_norm.restype = C.c_double
    L.or_norm.argtypes = [_dp, C.c_size_t]
    _lib = L
    return L


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def node_solve(a, c, d, e, g, bP, bU, bY):
    """eq. solution_reduced_system; returns (y, u, p)."""
    L = _load()
    N = len(a)
    y = np.zeros(N)
    p = np.zeros(N)
    u = C.c_double(0.0)
    L.or_node_solve(N, _f64(a), _f64(c), _f64(d), _f64(e), float(g), _f64(bP), float(bU),
                    _f64(bY), y, C.byref(u), p)
    return y, u.value, p


def restrict(nf: int, N: int, fine):
    nc = (nf - 1) // 2
    out = np.zeros((2 * N + 1) * nc * nc)
    _load().or_restrict(nf, N, _f64(fine), out)
    return out


def prolong_add(nc: int, N: int, coarse, fine):
    fine = _f64(fine).copy()
    _load().or_prolong_add(nc, N, _f64(coarse), fine)
    return fine


def coarsen_faces(nf: int, N: int, kx, ky):
    nc = (nf - 1) // 2
    kxc = np.zeros((N, nc, nc + 1))
    kyc = np.zeros((N, nc + 1, nc))
    _load().or_coarsen_faces(nf, N, _f64(kx), _f64(ky), kxc, kyc)
    return kxc, kyc


def num_threads() -> int:
    return int(_load().or_num_threads())


def norm(v) -> float:
    v = _f64(v)
    return _load().or_norm(v, v.size)


class Oracle:
    """Level hierarchy + coarsest factorization for one problem instance."""

    def __init__(self, prob, coarsest_n: int = 7, pre: int = 2, post: int = 2, theta: float = 1.0,
                 smoother: str = "gs"):
        """smoother: "gs" (red-black collective Gauss-Seidel sweeps) or "jacobi"
        (damped collective Jacobi steps, eq. collective_smoothing, damping theta)."""
        L = _load()
        self.n, self.N = prob.n, prob.N
        self.prob = prob
        if smoother not in ("gs", "jacobi"):
            raise ValueError("smoother must be 'gs' or 'jacobi'")
        self.ctx = L.or_create(prob.n, prob.N, coarsest_n, pre, post, theta, _f64(prob.kx),
                               _f64(prob.ky), _f64(prob.c), _f64(prob.d), _f64(prob.e),
                               float(prob.g))
        if not self.ctx:
            raise ValueError("oracle: invalid grid size or singular coarsest block")
        L.or_set_smoother(self.ctx, 1 if smoother == "jacobi" else 0)
        growth = float((getattr(prob, "meta", None) or {}).get("control_growth", 0.0))
        if growth and L.or_set_control_growth(self.ctx, growth) != 0:
            raise ValueError("oracle: singular coarsest block with this control growth")
        if getattr(prob, "domain", None) is not None:
            if L.or_set_domain(self.ctx, _f64(prob.domain)) != 0:
                raise ValueError("oracle: singular coarsest block with this domain")
        if getattr(prob, "ctrl", None) is not None:
            if L.or_set_control(self.ctx, _f64(prob.ctrl)) != 0:
                raise ValueError("oracle: singular coarsest block with this control mask")
        self.nlev = L.or_nlevels(self.ctx)
        self.levels_n = [L.or_level_n(self.ctx, l) for l in range(self.nlev)]

    def set_masks(self, md, me, coarsen: str = "injection"):
        """Node factors of D_j (md) and E_j (me), [n][n] arrays of the finest level or
        None for 1; coarse levels by injection or full weighting ("full"), coarsest
        factorization rebuilt."""
        if coarsen not in ("injection", "full"):
            raise ValueError("coarsen must be 'injection' or 'full'")
        keep = [None if m is None else _f64(np.asarray(m).reshape(self.n, self.n)) for m in (md, me)]
        ptr = [None if m is None else m.ctypes.data for m in keep]
        if _load().or_set_masks(self.ctx, ptr[0], ptr[1], 1 if coarsen == "full" else 0) != 0:
            raise ValueError("oracle: singular coarsest block with these node factors")

    def set_sample_c(self, c):
        """Per-sample C_j = c_j I of the finest level (c_j >= 0), coarse levels
        4^l c_j, coarsest factorization rebuilt."""
        if _load().or_set_sample_c(self.ctx, _f64(np.asarray(c, dtype=np.float64).reshape(self.N))) != 0:
            raise ValueError("oracle: negative c_j or singular coarsest block")

    def level_domain(self, l: int):
        """The domain of level l, [n_l][n_l] (1 inside, 0 outside)."""
        n = self.levels_n[l]
        out = np.zeros(n * n)
        _load().or_level_domain(self.ctx, l, out)
        return out.reshape(n, n)

    def level_factor(self, l: int, which: str = "d"):
        """The node factor md (which="d") or me ("e") of level l, [n_l][n_l]."""
        n = self.levels_n[l]
        out = np.zeros(n * n)
        _load().or_level_factor(self.ctx, l, 0 if which == "d" else 1, out)
        return out.reshape(n, n)

    def __del__(self):
        if getattr(self, "ctx", None):
            try:
                _load().or_destroy(self.ctx)
            except TypeError:   # interpreter shutdown: the module's globals are gone
                pass
            self.ctx = None

    def vlen(self, l: int = 0) -> int:
        n = self.levels_n[l]
        return (2 * self.N + 1) * n * n

    def rhs(self):
        return self.prob.rhs_paper()

    def level_faces(self, l: int):
        n = self.levels_n[l]
        kx = np.zeros((self.N, n, n + 1))
        ky = np.zeros((self.N, n + 1, n))
        _load().or_level_faces(self.ctx, l, kx, ky)
        return kx, ky

    def level_scalars(self, l: int):
        c = np.zeros(self.N); d = np.zeros(self.N); e = np.zeros(self.N)
        g = C.c_double(0.0)
        _load().or_level_scalars(self.ctx, l, c, d, e, C.byref(g))
        return c, d, e, g.value

    def apply(self, x, l: int = 0):
        out = np.zeros(self.vlen(l))
        _load().or_apply(self.ctx, l, _f64(x), out)
        return out

    def residual(self, x, f, l: int = 0):
        out = np.zeros(self.vlen(l))
        _load().or_residual(self.ctx, l, _f64(x), _f64(f), out)
        return out

    def residual_restrict(self, x, f, l: int = 0):
        """The coarse right-hand side of Alg. 1 from level l: R (f - S x), the U
        block restricted within the control space (nodes whose D and E factors
        are not both zero), zero outside the domain."""
        out = np.zeros(self.vlen(l + 1))
        _load().or_residual_restrict(self.ctx, l, _f64(x), _f64(f), out)
        return out

    def prolong_control(self, coarse, fine, l: int = 0):
        """fine (level l) + P coarse, the U block prolongated into the control
        space only."""
        fine = _f64(fine).copy()
        _load().or_prolong_control(self.ctx, l, _f64(coarse), fine)
        return fine

    def halfsweep(self, x, f, colour: int, l: int = 0, theta: float = 1.0):
        x = _f64(x).copy()
        _load().or_halfsweep(self.ctx, l, colour, theta, x, _f64(f))
        return x

    def halfsweep32(self, x, f, colour: int, l: int = 0, theta: float = 1.0):
        """The half-sweep in FP32 arithmetic (x, f rounded to FP32), widened back."""
        x = _f64(x).copy()
        _load().or_halfsweep32(self.ctx, l, colour, theta, x, _f64(f))
        return x

    def jacobi(self, x, f, theta: float, l: int = 0):
        x = _f64(x).copy()
        _load().or_jacobi(self.ctx, l, theta, x, _f64(f))
        return x

    def coarse_solve(self, F):
        out = np.zeros(self.vlen(self.nlev - 1))
        _load().or_coarse_solve(self.ctx, _f64(F), out)
        return out

    def vcycle(self, x, f, ncycles: int = 1):
        x = _f64(x).copy()
        _load().or_vcycle(self.ctx, x, _f64(f), ncycles)
        return x

    def vcycle32(self, x, f, ncycles: int = 1):
        x = _f64(x).copy()
        _load().or_vcycle32(self.ctx, x, _f64(f), ncycles)
        return x

    def solve_vcycle(self, f, tol: float = 1e-10, maxit: int = 200, x0=None):
        x = np.zeros(self.vlen()) if x0 is None else _f64(x0).copy()
        hist = np.zeros(maxit + 1)
        its = _load().or_solve_vcycle(self.ctx, x, _f64(f), tol, maxit, hist)
        k = its if its >= 0 else maxit
        return x, its, hist[:k + 1]

    def gmres(self, f, m: int = 30, tol: float = 1e-10, maxit: int = 300, prec32: bool = False,
              x0=None):
        x = np.zeros(self.vlen()) if x0 is None else _f64(x0).copy()
        hist = np.zeros(maxit + 1)
        its = _load().or_gmres(self.ctx, x, _f64(f), m, tol, maxit, int(prec32), hist)
        k = its if its >= 0 else maxit
        return x, its, hist[:k + 1]

    def solve_ir(self, f, tol: float = 1e-10, inner_tol: float = 1e-5, m: int = 30,
                 maxit: int = 50, x0=None):
        x = np.zeros(self.vlen()) if x0 is None else _f64(x0).copy()
        hist = np.zeros(maxit + 1)
        inner = C.c_int(0)
        its = _load().or_solve_ir(self.ctx, x, _f64(f), tol, inner_tol, m, maxit, hist,
                                  C.byref(inner))
        k = its if its >= 0 else maxit
        return x, its, inner.value, hist[:k + 1]

    def assemble(self, l: int = 0) -> np.ndarray:
        """Dense S of level l, probed column by column through the operator."""
        n = self.vlen(l)
        S = np.zeros((n, n))
        e = np.zeros(n)
        for q in range(n):
            e[:] = 0.0
            e[q] = 1.0
            S[:, q] = self.apply(e, l)
        return S
