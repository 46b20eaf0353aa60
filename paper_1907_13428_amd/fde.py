"""Thin Python binding of libfde.so (include/fde.h): argument marshalling only.

Every step of the operator applies, the preconditioner, the Krylov solve and
the ADMM iteration runs in the library's HIP kernels on the GPU; this module
only converts arguments (torch CUDA tensors -> device pointers, the current
HIP stream -> hipStream_t) and status codes -> exceptions.  The library must
be built (``python -m paper_1907_13428_amd.build``); nothing here falls back
to a CPU implementation.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfde.so")

FDE_OK, FDE_ENOTCONV = 0, 1
FDE_EINVAL, FDE_ENOMEM, FDE_EHIP, FDE_ENONFINITE = -1, -2, -3, -4
_STATUS = {0: "FDE_OK", 1: "FDE_ENOTCONV", -1: "FDE_EINVAL", -2: "FDE_ENOMEM", -3: "FDE_EHIP",
           -4: "FDE_ENONFINITE"}

EXPORTED = ["fde_validate", "fde_host_tables", "fde_host_diag_scaling", "fde_create", "fde_destroy", "fde_set_params", "fde_apply_A",
            "fde_apply_A_noalloc",
            "fde_apply_S", "fde_precond", "fde_krylov", "fde_minres", "fde_set_bounds", "fde_admm_solve", "fde_grad", "fde_time_pass",
            "fde_pass_timing", "fde_pass_stats",
            "fde_autotune", "fde_batch_create", "fde_batch_destroy", "fde_batch_solve", "fde_last_error",
            "fde_version"]

PASS_NAMES = ["xpass_B", "ypass_B", "xpass_BT", "ypass_BT", "pre_xfwd", "pre_yfwd", "pre_t_div", "pre_yinv",
              "pre_xinv"]


class FdeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nt", ctypes.c_int32), ("T", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("dplus", ctypes.POINTER(ctypes.c_double)), ("dminus", ctypes.POINTER(ctypes.c_double)),
                ("ctrl_sign", ctypes.c_double), ("psi_scaling", ctypes.c_int32), ("obj_weights", ctypes.c_int32),
                ("precond_fp32", ctypes.c_int32), ("alpha_t", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("delta", ctypes.c_double), ("rho", ctypes.c_double),
                ("ya", ctypes.c_double), ("yb", ctypes.c_double), ("ua", ctypes.c_double), ("ub", ctypes.c_double),
                ("krylov_tol", ctypes.c_double), ("krylov_maxit", ctypes.c_int32), ("tol_mode", ctypes.c_int32),
                ("admm_tol", ctypes.c_double), ("admm_maxit", ctypes.c_int32), ("pcg_cold_start", ctypes.c_int32),
                ("prox", ctypes.c_int32), ("prox_cy", ctypes.c_double), ("prox_cu", ctypes.c_double),
                ("precond_kind", ctypes.c_int32), ("krylov_solver", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("admm_iters", ctypes.c_int32), ("pcg_total", ctypes.c_int32), ("pcg_last", ctypes.c_int32),
                ("pcg_max", ctypes.c_int32), ("r_p", ctypes.c_double), ("r_y", ctypes.c_double),
                ("r_u", ctypes.c_double), ("J", ctypes.c_double), ("t_total", ctypes.c_double),
                ("t_pcg", ctypes.c_double), ("dual_inf", ctypes.c_double), ("t_rhs", ctypes.c_double),
                ("t_krylov", ctypes.c_double), ("t_update", ctypes.c_double), ("batched", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libfde.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(f"{LIB_PATH} is missing: build it with python -m paper_1907_13428_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        D = ctypes.POINTER(ctypes.c_double)
        L.fde_validate.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Params)]
        L.fde_host_tables.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Params), D, D, D, D, D, D]
        L.fde_host_diag_scaling.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Params), D]
        L.fde_create.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Params), P, ctypes.POINTER(P)]
        L.fde_destroy.argtypes = [P]
        L.fde_set_params.argtypes = [P, ctypes.POINTER(Params)]
        L.fde_apply_A.argtypes = [P, P, P, ctypes.c_int]
        L.fde_apply_A_noalloc.argtypes = [P, P, P, ctypes.c_int]
        L.fde_apply_S.argtypes = [P, P, P]
        L.fde_precond.argtypes = [P, P, P]
        L.fde_krylov.argtypes = [P, P, P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        L.fde_minres.argtypes = [P, P, P, P, P, P, P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        L.fde_set_bounds.argtypes = [P, P, P, P, P]
        L.fde_admm_solve.argtypes = [P, P, P, P, P, P, P, P, P, P, ctypes.POINTER(Stats)]
        L.fde_grad.argtypes = [P, P, P, P, P, ctypes.c_int, P, D, P]
        L.fde_time_pass.argtypes = [P, ctypes.c_int, ctypes.c_int, D, D]
        L.fde_autotune.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
        L.fde_pass_timing.argtypes = [P, ctypes.c_int]
        L.fde_pass_stats.argtypes = [P, D, ctypes.POINTER(ctypes.c_int32), D]
        PP = ctypes.POINTER(ctypes.c_void_p)
        L.fde_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(Problem), ctypes.POINTER(Params),
                                       ctypes.POINTER(P)]
        L.fde_batch_destroy.argtypes = [P]
        L.fde_batch_solve.argtypes = [P, ctypes.c_int, PP, PP, PP, PP, PP, PP, PP, PP, PP, ctypes.POINTER(Stats),
                                      ctypes.POINTER(ctypes.c_int32)]
        L.fde_last_error.restype = ctypes.c_char_p
        L.fde_version.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("fde_last_error", "fde_version"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status, allow_notconv=True):
    if status == FDE_OK or (allow_notconv and status == FDE_ENOTCONV):
        return status
    raise FdeError(status, lib().fde_last_error().decode())


def make_problem(nx, ny, nt, alpha, beta, *, T=1.0, dplus=None, dminus=None, ctrl_sign=1.0, psi_scaling=1,
                 obj_weights=0, precond_fp32=0, alpha_t=1.0):
    """Build the C problem struct; the coefficient arrays are kept alive on it."""
    import numpy as np

    p = Problem(nx=nx, ny=ny, nt=nt, T=T, alpha=alpha, beta=beta, ctrl_sign=ctrl_sign,
                psi_scaling=int(psi_scaling), obj_weights=int(obj_weights), precond_fp32=int(precond_fp32),
                alpha_t=alpha_t)
    keep = []
    for name, arr in (("dplus", dplus), ("dminus", dminus)):
        if arr is not None:
            a = np.ascontiguousarray(arr, dtype=np.float64)
            if a.size != nx * ny:
                raise ValueError(f"{name} must hold nx*ny values")
            keep.append(a)
            setattr(p, name, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    p._keep = keep
    return p


def make_params(gamma, *, delta=1.0, rho=1.0, ya=-math.inf, yb=math.inf, ua=-math.inf, ub=math.inf,
                krylov_tol=1e-10, krylov_maxit=1000, tol_mode=0, admm_tol=1e-6, admm_maxit=100000,
                pcg_cold_start=0, prox=0, prox_cy=0.0, prox_cu=0.0, precond_kind=0, krylov_solver=0):
    return Params(gamma=gamma, delta=delta, rho=rho, ya=ya, yb=yb, ua=ua, ub=ub, krylov_tol=krylov_tol,
                  krylov_maxit=krylov_maxit, tol_mode=tol_mode, admm_tol=admm_tol, admm_maxit=admm_maxit,
                  pcg_cold_start=pcg_cold_start, prox=prox, prox_cy=prox_cy, prox_cu=prox_cu,
                  precond_kind=precond_kind, krylov_solver=krylov_solver)


def from_workload(w, precond_fp32=0, **overrides):
    """(Problem, Params) from any object with the workload attributes."""
    prob = make_problem(w.nx, w.ny, w.nt, w.alpha, w.beta, T=w.T, dplus=w.dplus, dminus=w.dminus,
                        ctrl_sign=w.ctrl_sign, psi_scaling=w.psi_scaling, obj_weights=w.obj_weights,
                        precond_fp32=precond_fp32, alpha_t=getattr(w, "alpha_t", 1.0))
    kw = dict(delta=w.delta, rho=w.rho, ya=w.ya, yb=w.yb, ua=w.ua, ub=w.ub, krylov_tol=w.krylov_tol,
              krylov_maxit=w.krylov_maxit, admm_tol=w.admm_tol, admm_maxit=w.admm_maxit,
              tol_mode=getattr(w, "tol_mode", 0), pcg_cold_start=getattr(w, "pcg_cold_start", 0),
              prox=getattr(w, "prox", 0), prox_cy=getattr(w, "prox_cy", 0.0), prox_cu=getattr(w, "prox_cu", 0.0),
              precond_kind=getattr(w, "precond_kind", 0), krylov_solver=getattr(w, "krylov_solver", 0))
    kw.update(overrides)
    return prob, make_params(w.gamma, **kw)


def validate(prob, prm):
    return _check(lib().fde_validate(ctypes.byref(prob), ctypes.byref(prm)), allow_notconv=False)


def host_tables(prob, prm):
    """Host-only setup tables (no GPU use): scalars, T. Chan eigenvalues, weights."""
    import numpy as np

    scal = np.zeros(8)
    lx = np.zeros(2 * prob.nx)
    ly = np.zeros(2 * prob.ny)
    lt = np.zeros(2 * prob.nt)
    gx = np.zeros(prob.nx + 1)
    gy = np.zeros(prob.ny + 1)
    ptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib().fde_host_tables(ctypes.byref(prob), ctypes.byref(prm), ptr(scal), ptr(lx), ptr(ly), ptr(lt),
                                 ptr(gx), ptr(gy)), allow_notconv=False)
    c = lambda a: a[0::2] + 1j * a[1::2]
    keys = ["psi", "hx", "hy", "ht", "a", "inv_mbar", "e_u", "k_u"]
    return dict(zip(keys, scal.tolist()), lam_x=c(lx), lam_y=c(ly), lam_t=c(lt), gx=gx, gy=gy)


def host_diag_scaling(prob, prm):
    """fde_host_diag_scaling: the diagonal scaling Delta of precond_kind 2, as an
    (nt, ny, nx) array (host computation)."""
    import numpy as np

    out = np.zeros((prob.nt, prob.ny, prob.nx))
    _check(lib().fde_host_diag_scaling(ctypes.byref(prob), ctypes.byref(prm),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), allow_notconv=False)
    return out


def _dptr(t, name="tensor"):
    if t is None:
        return None
    import torch

    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """Owns an fde_ctx (device tables + workspace) bound to a HIP stream."""

    def __init__(self, prob: Problem, prm: Params, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("a GPU is required (libfde.so runs on gfx950)")
        self.prob, self.prm = prob, prm
        self.shape = (prob.nt, prob.ny, prob.nx)
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        h = ctypes.c_void_p()
        _check(lib().fde_create(ctypes.byref(prob), ctypes.byref(prm), ctypes.c_void_p(s.cuda_stream),
                                ctypes.byref(h)), allow_notconv=False)
        self._h = h

    # -- lifecycle -------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().fde_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_params(self, prm: Params):
        _check(lib().fde_set_params(self._h, ctypes.byref(prm)), allow_notconv=False)
        self.prm = prm

    # -- entry points ----------------------------------------------------
    def apply_A(self, x, y, transpose=False):
        _check(lib().fde_apply_A(self._h, _dptr(x, "x"), _dptr(y, "y"), int(transpose)), False)
        return y

    def apply_A_noalloc(self, x, y, transpose=False):
        """apply_A with the library's static per-GPU workspace (no device allocation)."""
        _check(lib().fde_apply_A_noalloc(self._h, _dptr(x, "x"), _dptr(y, "y"), int(transpose)), False)
        return y

    def apply_S(self, x, y):
        _check(lib().fde_apply_S(self._h, _dptr(x, "x"), _dptr(y, "y")), False)
        return y

    def precond(self, r, z):
        _check(lib().fde_precond(self._h, _dptr(r, "r"), _dptr(z, "z")), False)
        return z

    def krylov(self, b, x):
        it = ctypes.c_int()
        rel = ctypes.c_double()
        st = _check(lib().fde_krylov(self._h, _dptr(b, "b"), _dptr(x, "x"), ctypes.byref(it), ctypes.byref(rel)))
        return it.value, rel.value, st

    def minres(self, b, x):
        """MINRES on the merged x-step system: b and x are (y, u, p) tuples of
        device fields; x holds the initial guess and receives the solution.
        Returns (iterations, relative residual, status)."""
        it = ctypes.c_int()
        rel = ctypes.c_double()
        st = _check(lib().fde_minres(self._h, *(_dptr(f, n) for f, n in zip(b, ("b_y", "b_u", "b_p"))),
                                     *(_dptr(f, n) for f, n in zip(x, ("y", "u", "p"))), ctypes.byref(it),
                                     ctypes.byref(rel)))
        return it.value, rel.value, st

    def set_bounds(self, ya=None, yb=None, ua=None, ub=None):
        """Per-point box bounds (device fields of the grid's shape); None keeps
        the scalar bound of the parameters for that side."""
        for t, n in ((ya, "ya"), (yb, "yb"), (ua, "ua"), (ub, "ub")):
            if t is not None and tuple(t.shape) != tuple(self.shape):
                raise ValueError(f"{n} must have the grid's shape {tuple(self.shape)}")
        _check(lib().fde_set_bounds(self._h, _dptr(ya, "ya"), _dptr(yb, "yb"), _dptr(ua, "ua"), _dptr(ub, "ub")),
               False)

    def admm_solve(self, yhat, g=None, state=None):
        """Run ADMM; `state` = dict of y, u, zy, zu, p, wy, wu tensors (zeros if None),
        updated in place.  Returns (state, stats dict, status)."""
        import torch

        if state is None:
            state = {k: torch.zeros(self.shape, dtype=torch.float64, device=yhat.device)
                     for k in ("y", "u", "zy", "zu", "p", "wy", "wu")}
        st = Stats()
        args = [_dptr(state[k], k) for k in ("y", "u", "zy", "zu", "p", "wy", "wu")]
        status = _check(lib().fde_admm_solve(self._h, _dptr(yhat, "yhat"), _dptr(g, "g"), *args,
                                             ctypes.byref(st)))
        return state, st.as_dict(), status

    def autotune(self):
        """Pick the fastest column-tile variants for this grid; returns the choices."""
        ch = (ctypes.c_int32 * 3)()
        _check(lib().fde_autotune(self._h, ch), False)
        return list(ch)

    def time_pass(self, which, reps=20):
        """(mean microseconds per launch, algorithmic bytes per launch) of pass `which`."""
        us = ctypes.c_double()
        b = ctypes.c_double()
        _check(lib().fde_time_pass(self._h, int(which), int(reps), ctypes.byref(us), ctypes.byref(b)), False)
        return us.value, b.value

    def pass_timing(self, enable=True):
        """Time the nine PCG passes inside the following solves (plain launches, events per pass)."""
        _check(lib().fde_pass_timing(self._h, int(bool(enable))), False)

    def pass_stats(self):
        """{pass name: (mean us per launch, launches, algorithmic bytes per launch)} of the timed solves."""
        us = (ctypes.c_double * 9)()
        n = (ctypes.c_int32 * 9)()
        b = (ctypes.c_double * 9)()
        _check(lib().fde_pass_stats(self._h, us, n, b), False)
        return {name: (us[i], n[i], b[i]) for i, name in enumerate(PASS_NAMES)}

    def grad(self, yhat, y, p, wy=None, adjoint_solve=False, dyhat=None, lam=None):
        """(dJ/dyhat field, dJ/dalpha, dJ/dbeta) at an ADMM solution."""
        dab = (ctypes.c_double * 2)()
        _check(lib().fde_grad(self._h, _dptr(yhat), _dptr(y), _dptr(p), _dptr(wy), int(adjoint_solve),
                              _dptr(dyhat), dab, _dptr(lam)), False)
        return dyhat, dab[0], dab[1]


class Batch:
    """Many independent instances (uneven sizes) solved together: one context
    and stream per instance, driven concurrently by the library."""

    FIELDS = ("y", "u", "zy", "zu", "p", "wy", "wu")

    def __init__(self, probs, prms):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("a GPU is required (libfde.so runs on gfx950)")
        n = len(probs)
        self.count = n
        self.shapes = [(p.nt, p.ny, p.nx) for p in probs]
        self._probs = (Problem * n)(*probs)
        self._prms = (Params * n)(*prms)
        self._keep = [getattr(p, "_keep", None) for p in probs]
        h = ctypes.c_void_p()
        _check(lib().fde_batch_create(n, self._probs, self._prms, ctypes.byref(h)), allow_notconv=False)
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().fde_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def solve(self, yhats, states=None, concurrent=True, lockstep=False):
        """Solve every instance; returns (states, list of stats dicts, list of statuses).
        lockstep: all instances in step, their Krylov iterations as batched pass
        launches (falls back to the concurrent mode where that is unavailable)."""
        import torch

        n = self.count
        if states is None:
            states = [{k: torch.zeros(self.shapes[i], dtype=torch.float64, device="cuda") for k in self.FIELDS}
                      for i in range(n)]
        torch.cuda.synchronize()
        arr = lambda ts: (ctypes.c_void_p * n)(*[_dptr(t).value for t in ts])
        yh = arr(yhats)
        cols = [arr([states[i][k] for i in range(n)]) for k in self.FIELDS]
        st = (Stats * n)()
        code = (ctypes.c_int32 * n)()
        mode = 2 if lockstep else int(bool(concurrent))
        _check(lib().fde_batch_solve(self._h, mode, yh, None, *cols, st, code))
        return states, [s.as_dict() for s in st], list(code)
