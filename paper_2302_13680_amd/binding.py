"""Thin ctypes binding of libsmg.so (the C ABI of include/smg.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Device memory and the stream come from PyTorch (ROCm build); vectors and
faces are torch tensors in the library's node layout (samples innermost).
The binding refuses to run without the compiled library: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmg.so")

SMG_OK, SMG_NOT_CONVERGED = 0, 1
SMG_F64, SMG_F32 = 0, 1
SMG_VCYCLE, SMG_GMRES = 0, 1
SMG_FLAG_EAGER = 1
SMG_FLAG_UNFUSED = 2
SMG_FLAG_JACOBI = 4
SMG_FLAG_SSN = 8
SMG_FLAG_CVAR = 16
SMG_FLAG_HALFSWEEPS = 32
SMG_COARSEN_INJECT, SMG_COARSEN_FULL = 0, 1

EXPORTED = [
    "smg_workspace_bytes", "smg_setup", "smg_destroy", "smg_strerror", "smg_last_error",
    "smg_num_levels", "smg_level_n", "smg_apply", "smg_residual", "smg_residual_static", "smg_smooth", "smg_smooth32", "smg_sweep",
    "smg_sweep32", "smg_stream_copy", "smg_restrict",
    "smg_residual_restrict", "smg_residual_restrict_after_sweep", "smg_jacobi", "smg_prolong_add", "smg_coarse_solve", "smg_level_faces", "smg_vcycle", "smg_gmres_precond",
    "smg_solve", "smg_batch_workspace_bytes", "smg_batch_setup", "smg_batch_solve", "smg_batch_destroy",
    "smg_batch_last_error", "smg_tune_lanes", "smg_net_param_count", "smg_net_workspace_bytes",
    "smg_net_setup", "smg_net_destroy", "smg_net_last_error", "smg_net_set_params", "smg_net_get_params",
    "smg_net_forward", "smg_net_grad", "smg_net_train_step", "smg_net_features", "smg_net_targets",
    "smg_net_lift", "smg_set_node_factors", "smg_ssn_eval", "smg_ssn_merit", "smg_ssn_solve",
    "smg_set_sample_weights", "smg_set_lowrank", "smg_cvar_solve",
]


class Desc(C.Structure):
    _fields_ = [("n", C.c_int), ("nsamples", C.c_int), ("coarsest_n", C.c_int), ("pre", C.c_int),
                ("post", C.c_int), ("theta", C.c_double), ("precision", C.c_int),
                ("gmres_restart", C.c_int), ("flags", C.c_int), ("strip", C.c_int), ("sweep_rows", C.c_int)]


class Blocks(C.Structure):
    _fields_ = [("kx", C.c_void_p), ("ky", C.c_void_p), ("c", C.POINTER(C.c_double)),
                ("d", C.POINTER(C.c_double)), ("e", C.POINTER(C.c_double)), ("g", C.c_double),
                ("ctrl", C.POINTER(C.c_double)), ("domain", C.POINTER(C.c_double)),
                ("control_growth", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("inner_iterations", C.c_int), ("restarts", C.c_int),
                ("relres", C.c_double), ("relres_y", C.c_double), ("relres_u", C.c_double),
                ("relres_p", C.c_double), ("time_ms", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int),
                ("history_len", C.c_int)]


class SsnParams(C.Structure):
    _fields_ = [("nu", C.c_double), ("beta", C.c_double), ("a", C.c_double), ("b", C.c_double),
                ("mass", C.c_double), ("tol", C.c_double), ("inner_rtol", C.c_double),
                ("inner_method", C.c_int), ("maxit", C.c_int), ("inner_maxit", C.c_int),
                ("sigma", C.c_double), ("rho", C.c_double)]


class CvarParams(C.Structure):
    _fields_ = [("lam", C.c_double), ("eps", C.c_double), ("mass", C.c_double),
                ("zeta", C.POINTER(C.c_double)), ("tol", C.c_double), ("inner_tol", C.c_double),
                ("lin_rtol", C.c_double), ("maxit", C.c_int), ("inner_maxit", C.c_int),
                ("lin_maxit", C.c_int), ("sigma", C.c_double), ("rho", C.c_double),
                ("inner_rule", C.c_int), ("inner_full_steps", C.c_int)]


class CvarStats(C.Structure):
    _fields_ = [("outer", C.c_int), ("inner_total", C.c_int), ("linear_solves", C.c_int),
                ("linear_total", C.c_int), ("t", C.c_double), ("F_final", C.c_double),
                ("time_ms", C.c_double), ("F", C.POINTER(C.c_double)), ("cap", C.c_int), ("len", C.c_int),
                ("inner_capped", C.c_int), ("inner_stalled", C.c_int), ("inner_counts", C.POINTER(C.c_int)),
                ("inner_cap", C.c_int),
                ("inner_len", C.c_int)]


class SsnStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("inner_total", C.c_int), ("init_iterations", C.c_int),
                ("phi_final", C.c_double), ("time_ms", C.c_double), ("phi", C.POINTER(C.c_double)),
                ("gamma", C.POINTER(C.c_double)), ("inner", C.POINTER(C.c_int)), ("cap", C.c_int),
                ("len", C.c_int)]


def ssn_params(nu, beta, a, b, mass, *, tol=1e-9, inner_rtol=1e-11, inner_method=SMG_GMRES, maxit=100,
               inner_maxit=500, sigma=1e-4, rho=0.5):
    """smg_ssn_params (Section 5, Algorithm 2); a, b may be -inf / inf."""
    return SsnParams(float(nu), float(beta), float(a), float(b), float(mass), float(tol), float(inner_rtol),
                     int(inner_method), int(maxit), int(inner_maxit), float(sigma), float(rho))


class SmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"smg error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libsmg.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2302_13680_amd.build.build()")
    # The PyTorch ROCm wheel carries its own HIP runtime.  Loaded first, it is
    # the runtime the library binds to, so the streams and device pointers torch
    # hands over belong to the runtime the library calls; loaded after the
    # library, a second runtime would come in beside the system one and every
    # call on torch's memory would fail.
    import torch  # noqa: F401
    L = C.CDLL(path)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    L.smg_workspace_bytes.restype = C.c_size_t
    L.smg_workspace_bytes.argtypes = [C.POINTER(Desc)]
    L.smg_setup.restype = i
    L.smg_setup.argtypes = [C.POINTER(Desc), C.POINTER(Blocks), vp, C.c_size_t, vp, C.POINTER(vp)]
    L.smg_destroy.argtypes = [vp]
    L.smg_strerror.restype = C.c_char_p
    L.smg_strerror.argtypes = [i]
    L.smg_last_error.restype = C.c_char_p
    L.smg_last_error.argtypes = [vp]
    L.smg_num_levels.argtypes = [vp]
    L.smg_level_n.argtypes = [vp, i]
    L.smg_apply.argtypes = [vp, vp, vp]
    L.smg_residual.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_double)]
    L.smg_residual_static.argtypes = [vp, vp, vp, vp, vp]
    L.smg_smooth.argtypes = [vp, i, i, vp, vp]
    L.smg_smooth32.argtypes = [vp, i, i, vp, vp]
    L.smg_sweep.argtypes = [vp, i, vp, vp, vp, C.POINTER(i)]
    L.smg_sweep32.argtypes = [vp, i, vp, vp, vp, C.POINTER(i)]
    L.smg_stream_copy.argtypes = [vp, vp, C.c_size_t, vp]
    L.smg_stream_copy.restype = i
    L.smg_restrict.argtypes = [vp, i, vp, vp]
    L.smg_residual_restrict.argtypes = [vp, i, vp, vp, vp]
    L.smg_residual_restrict_after_sweep.argtypes = [vp, i, vp, vp, vp, vp, C.POINTER(i)]
    L.smg_jacobi.argtypes = [vp, i, vp, vp, vp]
    L.smg_prolong_add.argtypes = [vp, i, vp, vp]
    L.smg_coarse_solve.argtypes = [vp, vp, vp]
    L.smg_level_faces.argtypes = [vp, i, vp, vp]
    L.smg_vcycle.argtypes = [vp, vp, vp, i]
    L.smg_gmres_precond.argtypes = [vp, vp, vp, i, d, i, C.POINTER(Stats)]
    L.smg_solve.argtypes = [vp, vp, vp, i, d, i, C.POINTER(Stats)]
    L.smg_batch_workspace_bytes.restype = C.c_size_t
    L.smg_batch_workspace_bytes.argtypes = [C.POINTER(vp), i]
    L.smg_batch_setup.restype = i
    L.smg_batch_setup.argtypes = [C.POINTER(vp), i, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int), vp,
                                  C.c_size_t, C.POINTER(vp)]
    L.smg_batch_solve.restype = i
    L.smg_batch_solve.argtypes = [vp, d, i, C.POINTER(Stats), C.POINTER(C.c_double)]
    L.smg_batch_destroy.argtypes = [vp]
    L.smg_batch_last_error.restype = C.c_char_p
    L.smg_batch_last_error.argtypes = [vp]
    L.smg_tune_lanes.restype = i
    L.smg_tune_lanes.argtypes = [vp, i, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_int),
                                 C.POINTER(C.c_int)]
    fp = C.POINTER(C.c_float)
    L.smg_net_param_count.restype = i
    L.smg_net_workspace_bytes.restype = C.c_size_t
    L.smg_net_workspace_bytes.argtypes = [i, i]
    L.smg_net_setup.restype = i
    L.smg_net_setup.argtypes = [i, i, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.smg_net_destroy.argtypes = [vp]
    L.smg_net_last_error.restype = C.c_char_p
    L.smg_net_last_error.argtypes = [vp]
    L.smg_net_set_params.argtypes = [vp, vp]
    L.smg_net_get_params.argtypes = [vp, vp]
    L.smg_net_forward.argtypes = [vp, vp, vp]
    L.smg_net_grad.argtypes = [vp, vp, vp, i, vp, fp]
    L.smg_net_train_step.argtypes = [vp, vp, vp, i, C.c_float, fp]
    L.smg_net_features.argtypes = [vp, vp, i, vp]
    L.smg_net_targets.argtypes = [vp, vp, i, fp, vp]
    L.smg_net_lift.argtypes = [vp, vp, i, fp, vp]
    for name in ["smg_net_set_params", "smg_net_get_params", "smg_net_forward", "smg_net_grad",
                 "smg_net_train_step", "smg_net_features", "smg_net_targets", "smg_net_lift"]:
        getattr(L, name).restype = i
    L.smg_set_node_factors.argtypes = [vp, vp, vp, i]
    L.smg_ssn_eval.argtypes = [vp, vp, C.POINTER(SsnParams), vp, vp, vp, C.POINTER(C.c_double)]
    L.smg_ssn_merit.argtypes = [vp, vp, vp, vp, vp, C.POINTER(SsnParams), i, C.POINTER(C.c_double),
                                C.POINTER(C.c_double)]
    L.smg_ssn_solve.argtypes = [vp, vp, vp, C.POINTER(SsnParams), C.POINTER(SsnStats)]
    for name in ["smg_set_node_factors", "smg_ssn_eval", "smg_ssn_merit", "smg_ssn_solve"]:
        getattr(L, name).restype = i
    L.smg_set_sample_weights.argtypes = [vp, C.POINTER(C.c_double)]
    L.smg_set_lowrank.argtypes = [vp, vp, vp]
    L.smg_cvar_solve.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_double), C.POINTER(CvarParams),
                                 C.POINTER(CvarStats)]
    for name in ["smg_set_sample_weights", "smg_set_lowrank", "smg_cvar_solve"]:
        getattr(L, name).restype = i
    for name in ["smg_apply", "smg_residual", "smg_smooth", "smg_smooth32", "smg_stream_copy", "smg_restrict", "smg_residual_restrict",
                 "smg_residual_restrict_after_sweep", "smg_jacobi", "smg_prolong_add",
                 "smg_coarse_solve", "smg_level_faces", "smg_vcycle", "smg_gmres_precond", "smg_solve",
                 "smg_num_levels", "smg_level_n"]:
        getattr(L, name).restype = i
    _lib = L
    return L


def _ptr(t):
    import torch
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return C.c_void_p(t.data_ptr())


def workspace_bytes(n, N, coarsest_n=7, pre=2, post=2, theta=1.0, precision=SMG_F64, gmres_restart=30,
                    flags=0, strip=0, sweep_rows=0):
    L = load()
    desc = Desc(n, N, coarsest_n, pre, post, theta, precision, gmres_restart, flags, strip, sweep_rows)
    return int(L.smg_workspace_bytes(C.byref(desc)))


class Context:
    """One smg_ctx: hierarchy + coarsest factorization for one instance.

    kx, ky: float64 device tensors in the node layout ([n][n+1][N], [n+1][n][N]);
    c, d, e: per-sample diagonal values (host sequences), g: scalar; ctrl: optional
    (n, n) host control mask in [0, 1] (local control), None: control everywhere; domain:
    optional (n, n) host 0/1 mask of the domain (the L-shape), None: the square;
    control_growth: per-coarsening factor of d, e, g (0: 4; 2 for a control on a line).
    """

    def __init__(self, n, N, kx, ky, c, d, e, g, *, coarsest_n=7, pre=2, post=2, theta=1.0,
                 precision=SMG_F64, gmres_restart=30, flags=0, strip=0, stream=None, ctrl=None, domain=None,
                 control_growth=0.0, sweep_rows=0):
        import torch
        L = load()
        self.L = L
        self.n, self.N = n, N
        self.precision = precision
        self.device = kx.device
        self.desc = Desc(n, N, coarsest_n, pre, post, theta, precision, gmres_restart, flags, strip, sweep_rows)
        nbytes = int(L.smg_workspace_bytes(C.byref(self.desc)))
        if nbytes == 0:
            raise SmgError(-1, "invalid descriptor")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.kx, self.ky = kx, ky     # referenced by the library: keep alive
        self._c = np.ascontiguousarray(c, dtype=np.float64)
        self._d = np.ascontiguousarray(d, dtype=np.float64)
        self._e = np.ascontiguousarray(e, dtype=np.float64)
        dp = C.POINTER(C.c_double)
        self._ctrl = None if ctrl is None else np.ascontiguousarray(ctrl, dtype=np.float64).reshape(n * n)
        self._dom = None if domain is None else np.ascontiguousarray(domain, dtype=np.float64).reshape(n * n)
        blocks = Blocks(_ptr(kx), _ptr(ky), self._c.ctypes.data_as(dp), self._d.ctypes.data_as(dp),
                        self._e.ctypes.data_as(dp), float(g),
                        None if self._ctrl is None else self._ctrl.ctypes.data_as(dp),
                        None if self._dom is None else self._dom.ctypes.data_as(dp), float(control_growth))
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        rc = L.smg_setup(C.byref(self.desc), C.byref(blocks), _ptr(self.workspace), nbytes,
                         C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if rc != SMG_OK:
            raise SmgError(rc, L.smg_strerror(rc).decode())
        self.ctx = ctx
        self.nlev = L.smg_num_levels(ctx)
        self.levels_n = [L.smg_level_n(ctx, l) for l in range(self.nlev)]

    def close(self):
        if getattr(self, "ctx", None):
            self.L.smg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_nc=False):
        if rc == SMG_OK or (allow_nc and rc == SMG_NOT_CONVERGED):
            return rc
        detail = self.L.smg_last_error(self.ctx).decode() if self.ctx else ""
        raise SmgError(rc, self.L.smg_strerror(rc).decode() + (": " + detail if detail else ""))

    def vlen(self, level=0):
        n = self.levels_n[level]
        return (2 * self.N + 1) * n * n

    # --- steps ------------------------------------------------------------
    def apply(self, x, out):
        return self._check(self.L.smg_apply(self.ctx, _ptr(x), _ptr(out)))

    def residual(self, x, f, r, norms=False):
        if norms:
            buf = (C.c_double * 4)()
            self._check(self.L.smg_residual(self.ctx, _ptr(x), _ptr(f), _ptr(r), buf))
            return list(buf)
        self._check(self.L.smg_residual(self.ctx, _ptr(x), _ptr(f), _ptr(r), None))
        return None

    def residual_static(self, x, f, r, norms_dev):
        """r = f - S x with the five norms written to the device tensor norms_dev
        (float64, 5 entries), partial sums in the library's static scratch."""
        return self._check(self.L.smg_residual_static(self.ctx, _ptr(x), _ptr(f), _ptr(r), _ptr(norms_dev)))

    def smooth(self, level, colour, x, f):
        return self._check(self.L.smg_smooth(self.ctx, level, colour, _ptr(x), _ptr(f)))

    def sweep(self, level, xin, xout, f):
        """One red+black sweep xin -> xout (FP64 contexts); returns True where it
        ran as one launch."""
        one = C.c_int(0)
        self._check(self.L.smg_sweep(self.ctx, level, _ptr(xin), _ptr(xout), _ptr(f), C.byref(one)))
        return bool(one.value)

    def sweep32(self, level, xin, xout, f):
        """The FP32 sweep on float32 device vectors (SMG_F32 contexts)."""
        one = C.c_int(0)
        self._check(self.L.smg_sweep32(self.ctx, level, _ptr(xin), _ptr(xout), _ptr(f), C.byref(one)))
        return bool(one.value)

    def smooth32(self, level, colour, x, f):
        """FP32 half-sweep on float32 device vectors (SMG_F32 contexts)."""
        return self._check(self.L.smg_smooth32(self.ctx, level, colour, _ptr(x), _ptr(f)))

    def restrict(self, level, fine, coarse):
        return self._check(self.L.smg_restrict(self.ctx, level, _ptr(fine), _ptr(coarse)))

    def jacobi(self, level, x, xout, f):
        return self._check(self.L.smg_jacobi(self.ctx, level, _ptr(x), _ptr(xout), _ptr(f)))

    def residual_restrict(self, level, x, f, coarse):
        return self._check(self.L.smg_residual_restrict(self.ctx, level, _ptr(x), _ptr(f), _ptr(coarse)))

    def residual_restrict_after_sweep(self, level, xold, xnew, f, coarse):
        """coarse = R (f - S xnew) for xnew one sweep of xold; returns True where it
        was formed from the blacks' change (f not read)."""
        fc = C.c_int(0)
        self._check(self.L.smg_residual_restrict_after_sweep(self.ctx, level, _ptr(xold), _ptr(xnew), _ptr(f),
                                                             _ptr(coarse), C.byref(fc)))
        return bool(fc.value)

    def prolong_add(self, level, coarse, fine):
        return self._check(self.L.smg_prolong_add(self.ctx, level, _ptr(coarse), _ptr(fine)))

    def coarse_solve(self, F, X):
        return self._check(self.L.smg_coarse_solve(self.ctx, _ptr(F), _ptr(X)))

    def level_faces(self, level, kx, ky):
        return self._check(self.L.smg_level_faces(self.ctx, level, _ptr(kx), _ptr(ky)))

    def vcycle(self, x, f, ncycles=1):
        return self._check(self.L.smg_vcycle(self.ctx, _ptr(x), _ptr(f), ncycles))

    def _stats(self, history):
        st = Stats()
        if history:
            self._hist = (C.c_double * history)()
            st.history = self._hist
            st.history_cap = history
        return st

    def gmres(self, x, f, restart=30, rtol=1e-10, maxit=200, history=256):
        st = self._stats(history)
        rc = self._check(self.L.smg_gmres_precond(self.ctx, _ptr(x), _ptr(f), restart, rtol, maxit,
                                                  C.byref(st)), allow_nc=True)
        return rc, _stats_dict(st)

    def solve(self, x, f, method=SMG_VCYCLE, rtol=1e-10, maxit=200, history=256):
        st = self._stats(history)
        rc = self._check(self.L.smg_solve(self.ctx, _ptr(x), _ptr(f), method, rtol, maxit, C.byref(st)),
                         allow_nc=True)
        return rc, _stats_dict(st)

    # --- node factors and the semismooth Newton solver ----------------------
    def set_node_factors(self, md=None, me=None, coarsening=SMG_COARSEN_INJECT):
        """md, me: float64 device tensors [n][n] (or None for 1)."""
        return self._check(self.L.smg_set_node_factors(
            self.ctx, None if md is None else _ptr(md), None if me is None else _ptr(me), int(coarsening)))

    def ssn_eval(self, x, prm, w, F=None, chi=None):
        """w = E[p] per node; with F, chi also F(u), the active set and the merit (returned)."""
        phi = C.c_double(0.0)
        self._check(self.L.smg_ssn_eval(self.ctx, _ptr(x), C.byref(prm), _ptr(w),
                                        None if F is None else _ptr(F), None if chi is None else _ptr(chi),
                                        C.byref(phi)))
        return phi.value

    def ssn_merit(self, u, du, w, dw, prm, gammas):
        ng = len(gammas)
        g = (C.c_double * ng)(*[float(v) for v in gammas])
        out = (C.c_double * ng)()
        self._check(self.L.smg_ssn_merit(self.ctx, _ptr(u), _ptr(du), _ptr(w), _ptr(dw), C.byref(prm), ng, g, out))
        return list(out)

    def ssn_solve(self, x, f, prm, cap=256):
        """Algorithm 2 in place on x (its U block: u^0).  Returns (rc, stats dict)."""
        phi = (C.c_double * cap)()
        gam = (C.c_double * cap)()
        inner = (C.c_int * cap)()
        st = SsnStats(0, 0, 0, 0.0, 0.0, phi, gam, inner, cap, 0)
        rc = self._check(self.L.smg_ssn_solve(self.ctx, _ptr(x), _ptr(f), C.byref(prm), C.byref(st)),
                         allow_nc=True)
        k = min(st.len, cap)
        return rc, dict(iterations=st.iterations, inner_total=st.inner_total,
                        init_iterations=st.init_iterations, phi_final=st.phi_final, time_ms=st.time_ms,
                        phi=list(phi[:k]), gammas=list(gam[:max(k - 1, 0)]), inner=list(inner[:max(k - 1, 0)]))

    def set_sample_weights(self, c):
        """C_j = c_j I on the finest level (host sequence of N values >= 0)."""
        self._cw = np.ascontiguousarray(c, dtype=np.float64)
        return self._check(self.L.smg_set_sample_weights(self.ctx, self._cw.ctypes.data_as(C.POINTER(C.c_double))))

    def set_lowrank(self, z, w):
        """Rank-one terms w_j z_j z_j^T (device tensors z [n][n][N], w [N]); None clears."""
        return self._check(self.L.smg_set_lowrank(self.ctx, None if z is None else _ptr(z),
                                                  None if w is None else _ptr(w)))

    def cvar_solve(self, x, f, yd, zeta, lam, eps, mass, t0=0.0, tol=1e-6, inner_tol=1e-8, lin_rtol=1e-9,
                   maxit=50, inner_maxit=50, lin_maxit=80, cap=256, inner_rule="max", inner_backtrack=True):
        """Algorithm 3 in place on x (device); yd: device [n][n].  inner_rule "max"
        (the printed rule) or "min"; inner_backtrack: the line search of the
        Newton steps for h(t) (False: full steps).  Returns (rc, stats dict)."""
        if inner_rule not in ("max", "min"):
            raise ValueError("inner_rule must be 'max' or 'min'")
        zeta = np.ascontiguousarray(zeta, dtype=np.float64)
        prm = CvarParams(lam, eps, mass, zeta.ctypes.data_as(C.POINTER(C.c_double)), tol, inner_tol, lin_rtol,
                         maxit, inner_maxit, lin_maxit, 0.0, 0.0, 1 if inner_rule == "min" else 0,
                         0 if inner_backtrack else 1)
        F = (C.c_double * cap)()
        counts = (C.c_int * cap)()
        st = CvarStats(0, 0, 0, 0, 0.0, 0.0, 0.0, F, cap, 0, 0, 0, counts, cap, 0)
        t = C.c_double(t0)
        rc = self._check(self.L.smg_cvar_solve(self.ctx, _ptr(x), _ptr(f), _ptr(yd), C.byref(t), C.byref(prm),
                                               C.byref(st)), allow_nc=True)
        return rc, dict(outer=st.outer, inner_total=st.inner_total, linear_solves=st.linear_solves,
                        linear_total=st.linear_total, t=t.value, F_final=st.F_final, time_ms=st.time_ms,
                        F=list(F[:min(st.len, cap)]), inner_capped=st.inner_capped,
                        inner_stalled=st.inner_stalled,
                        inner_counts=list(counts[:min(st.inner_len, cap)]))


class Batch:
    """smg_batch over several Contexts with bound FP64 device vectors x[i], f[i]."""

    def __init__(self, contexts, xs, fs, lanes=None):
        import torch
        L = load()
        self.L = L
        self.contexts = list(contexts)
        self.xs, self.fs = list(xs), list(fs)
        cnt = len(self.contexts)
        ctxs = (C.c_void_p * cnt)(*[c.ctx for c in self.contexts])
        nbytes = int(L.smg_batch_workspace_bytes(ctxs, cnt))
        if nbytes == 0:
            raise SmgError(-1, "invalid batch")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.contexts[0].device)
        xp = (C.c_void_p * cnt)(*[_ptr(x).value for x in self.xs])
        fp = (C.c_void_p * cnt)(*[_ptr(f).value for f in self.fs])
        lp = (C.c_int * cnt)(*lanes) if lanes is not None else None
        out = C.c_void_p()
        rc = L.smg_batch_setup(ctxs, cnt, xp, fp, lp, _ptr(self.workspace), nbytes, C.byref(out))
        if rc != SMG_OK:
            raise SmgError(rc, L.smg_strerror(rc).decode())
        self.batch = out
        self.lanes = list(lanes) if lanes is not None else None

    def solve(self, rtol=1e-8, maxit=100):
        cnt = len(self.contexts)
        st = (Stats * cnt)()
        wall = C.c_double(0.0)
        rc = self.L.smg_batch_solve(self.batch, rtol, maxit, st, C.byref(wall))
        if rc not in (SMG_OK, SMG_NOT_CONVERGED):
            raise SmgError(rc, self.L.smg_strerror(rc).decode() + ": " +
                           self.L.smg_batch_last_error(self.batch).decode())
        return rc, [_stats_dict(s) for s in st], wall.value

    def close(self):
        if getattr(self, "batch", None):
            self.L.smg_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stream_copy(dst, src, stream=None):
    """Copy src into dst (same byte size, device tensors) with the library's plain
    streaming kernel on `stream` (default: the current stream)."""
    import torch
    L = load()
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    rc = L.smg_stream_copy(_ptr(dst), _ptr(src), nbytes, C.c_void_p(s.cuda_stream))
    if rc != SMG_OK:
        raise SmgError(rc, L.smg_strerror(rc).decode())


def tune_lanes(ctx):
    """Time the batched half-sweep of one context for each lane width; returns
    (best_width, {width: microseconds})."""
    L = load()
    lanes = (C.c_int * 8)()
    us = (C.c_double * 8)()
    nc = C.c_int(0)
    best = C.c_int(0)
    rc = L.smg_tune_lanes(ctx.ctx, 8, lanes, us, C.byref(nc), C.byref(best))
    if rc != SMG_OK:
        raise SmgError(rc, L.smg_strerror(rc).decode())
    return best.value, {lanes[i]: us[i] for i in range(nc.value)}


class Net:
    """smg_net: the warm-start network for mini-batches of `batch` samples on H x H."""

    def __init__(self, batch, H, device="cuda", stream=None):
        import torch
        L = load()
        self.L, self.B, self.H = L, batch, H
        self.np = int(L.smg_net_param_count())
        nbytes = int(L.smg_net_workspace_bytes(batch, H))
        if nbytes == 0:
            raise SmgError(-1, "invalid network shape")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        out = C.c_void_p()
        rc = L.smg_net_setup(batch, H, _ptr(self.workspace), nbytes, C.c_void_p(self.stream.cuda_stream),
                             C.byref(out))
        if rc != SMG_OK:
            raise SmgError(rc, L.smg_strerror(rc).decode())
        self.net = out

    def _check(self, rc):
        if rc != SMG_OK:
            raise SmgError(rc, self.L.smg_strerror(rc).decode() + ": " + self.L.smg_net_last_error(self.net).decode())

    def set_params(self, theta):
        self._check(self.L.smg_net_set_params(self.net, _ptr(theta)))

    def get_params(self, out):
        self._check(self.L.smg_net_get_params(self.net, _ptr(out)))

    def forward(self, x, out):
        self._check(self.L.smg_net_forward(self.net, _ptr(x), _ptr(out)))

    def grad(self, x, target, valid, grad=None):
        loss = C.c_float(0.0)
        self._check(self.L.smg_net_grad(self.net, _ptr(x), _ptr(target), valid,
                                        _ptr(grad) if grad is not None else None, C.byref(loss)))
        return loss.value

    def train_step(self, x, target, valid, lr, want_loss=True):
        loss = C.c_float(0.0)
        self._check(self.L.smg_net_train_step(self.net, _ptr(x), _ptr(target), valid, float(lr),
                                              C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "net", None):
            self.L.smg_net_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def net_features(ctx, f, H, out):
    ctx._check(ctx.L.smg_net_features(ctx.ctx, _ptr(f), H, _ptr(out)))


def net_targets(ctx, x, H, norm, out):
    arr = (C.c_float * 6)(*[float(v) for v in norm])
    ctx._check(ctx.L.smg_net_targets(ctx.ctx, _ptr(x), H, arr, _ptr(out)))


def net_lift(ctx, pred, H, norm, x0):
    arr = (C.c_float * 6)(*[float(v) for v in norm])
    ctx._check(ctx.L.smg_net_lift(ctx.ctx, _ptr(pred), H, arr, _ptr(x0)))


def _stats_dict(st):
    hist = [st.history[i] for i in range(st.history_len)] if st.history_len else []
    return dict(iterations=st.iterations, inner_iterations=st.inner_iterations, restarts=st.restarts,
                relres=st.relres, relres_y=st.relres_y, relres_u=st.relres_u, relres_p=st.relres_p,
                time_ms=st.time_ms, history=hist)


def context_from_problem(prob, device="cuda", ssn=False, **kw):
    """Upload a problem's faces (node layout) and build a Context; returns (ctx, f).

    ssn=True builds the semismooth Newton solver's context instead: the Newton
    system's U row as printed (G = M, D_j / nu: the linear-quadratic row divided
    by nu) and SMG_FLAG_SSN."""
    import torch
    kxn, kyn = prob.faces_node()
    kx = torch.from_numpy(kxn).to(device)
    ky = torch.from_numpy(kyn).to(device)
    kw.setdefault("ctrl", getattr(prob, "ctrl", None))
    kw.setdefault("domain", getattr(prob, "domain", None))
    kw.setdefault("control_growth", float((getattr(prob, "meta", None) or {}).get("control_growth", 0.0)))
    g, d = prob.g, prob.d
    if ssn:
        g, d = prob.g / prob.nu, np.asarray(prob.d) / prob.nu
        kw["flags"] = kw.get("flags", 0) | SMG_FLAG_SSN
    ctx = Context(prob.n, prob.N, kx, ky, prob.c, d, prob.e, g, **kw)
    f = torch.from_numpy(prob.rhs_node()).to(device)
    return ctx, f
