"""Algorithm 1 (2-block standard ADMM) with the merged x-step -- oracle, test infrastructure.

Sec. 3.1.  With the constraints scaled as in Sec. 5/6.1 (B = psi D, the control
coupling k_u = psi * s with s = +-1, and the copy constraints on u scaled by
e_u = psi; e_y = 1), one iteration j is:

  1. R_y = rho (J1 yhat - e_y w_y + e_y^2 z_y / delta) + (1 - rho) B^T p
     R_u = rho (-e_u w_u + e_u^2 z_u / delta) + (1 - rho) k_u p
     M_y = rho (J1 + e_y^2/delta), M_u = rho (J2 + e_u^2/delta),
     M_p = k_u^2 M_u^{-1} + (delta/rho) I                (all diagonal)
     r   = k_u M_u^{-1} R_u - h + (delta/rho) p,   h = psi g
  2. S y = R_y - B^T M_p^{-1} r,  S = M_y + B^T M_p^{-1} B   (eq. (3.9))
  3. p = M_p^{-1}(B y + r),  u = M_u^{-1}(R_u - k_u p)
  4. z_y = Proj_[ya,yb](y + delta w_y / e_y), z_u = Proj_[ua,ub](u + delta w_u / e_u)
  5. w_y += (rho/delta) e_y (y - z_y),  w_u += (rho/delta) e_u (u - z_u)
  6. stop when max(|B y + k_u u - h|_inf, |y - z_y|_inf, |u - z_u|_inf) <= tol

Algorithm 2 (generalized ADMM, Sec. 3.3.2) adds the proximal term
1/2 (y - y^j)^T R_y (y - y^j) + 1/2 (u - u^j)^T R_u (u - u^j) to the x-step,
with R_y = c_y I - J1 and R_u = c_u I - J2.  It enters beside J1 and J2 under
the same factor rho, so the (1,1) and (2,2) blocks become the scaled
identities rho (c_y + e_y^2/delta) I and rho (c_u + e_u^2/delta) I (the
printed coefficient matrix of the generalized x-step), and step 1 gains
rho R_y y^j in R_y and rho R_u u^j in R_u.  The printed algorithm omits the
1/2 on the u term; the printed coefficient matrix fixes it.

Steps 1-3 are the elimination of u and p from the merged system (3.8); the
sign of the M_u^{-1} term in r is "+" (eliminating u from the third block row
gives + k_u M_u^{-1} R_u; the printed "-" does not reproduce the block solve,
which tests/test_oracle_admm.py checks).  Step 4 is the closed form of the
z-subproblem (3.6b); step 5 is (3.6d); p is updated inside step 3, which is
(3.6c) merged into the x-step.  The normal equations are solved by textbook
PCG (Sec. 6.1 uses MATLAB pcg) with the preconditioner S~ of eq. (3.10).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from . import operator as op
from .precond import apply_precond, apply_precond_scaled, diag_S, precond_tables, scaling_factor


@dataclasses.dataclass
class Scalars:
    psi: float
    e_y: float
    e_u: float
    k_u: float
    wts: np.ndarray  # (nt,) diagonal of J1 per time slice
    My: np.ndarray  # (nt,)
    Mu: np.ndarray  # (nt,)
    Mp: np.ndarray  # (nt,)
    cy: float = 0.0  # Algorithm 2 constants (0 under Algorithm 1)
    cu: float = 0.0


def objective_weights(w) -> np.ndarray:
    """J1 = diag(wts) (x) I: all ones, or trapezoidal with 1/2 on the last
    time block (eq. (4.10))."""
    wts = np.ones(w.nt)
    if w.obj_weights == 1:
        wts[-1] = 0.5
    return wts


def prox_constants(w, wts):
    """c_y, c_u of Algorithm 2 (Sec. 3.3.2).  The algorithm asks for R_y, R_u
    positive definite; c = max diag J (R semi-definite, zero where J is at its
    maximum) is accepted too and is what 0 selects."""
    cy = w.prox_cy if w.prox_cy > 0 else float(np.max(wts))
    cu = w.prox_cu if w.prox_cu > 0 else w.gamma * float(np.max(wts))
    return cy, cu


def scalars(w, d: op.Disc) -> Scalars:
    psi = op.psi_scale(d) if w.psi_scaling else 1.0
    e_y = 1.0
    e_u = psi if w.psi_scaling == 1 else 1.0
    k_u = psi * w.ctrl_sign
    wts = objective_weights(w)
    cy = cu = 0.0
    if getattr(w, "prox", 0):
        # Algorithm 2: J1 + R_y = c_y I, J2 + R_u = c_u I
        cy, cu = prox_constants(w, wts)
        My = w.rho * (cy + e_y ** 2 / w.delta) * np.ones(w.nt)
        Mu = w.rho * (cu + e_u ** 2 / w.delta) * np.ones(w.nt)
    else:
        My = w.rho * (wts + e_y ** 2 / w.delta)
        Mu = w.rho * (w.gamma * wts + e_u ** 2 / w.delta)
    Mp = k_u ** 2 / Mu + w.delta / w.rho
    return Scalars(psi, e_y, e_u, k_u, wts, My, Mu, Mp, cy, cu)


def tcol(a):
    """Broadcast a per-time-slice vector over (nt, ny, nx)."""
    return np.asarray(a)[:, None, None]


def apply_B(d, sc, v):
    return sc.psi * op.apply_D(d, v)


def apply_BT(d, sc, v):
    return sc.psi * op.apply_DT(d, v)


def apply_S(d, sc, v):
    """S v = M_y v + B^T M_p^{-1} B v (eq. (3.9), scaled form)."""
    return tcol(sc.My) * v + apply_BT(d, sc, apply_B(d, sc, v) / tcol(sc.Mp))


def pcg(A, M, b, x0, tol, maxit):
    """Textbook preconditioned CG (Fletcher-Reeves beta), stopping on the
    recursively updated residual: ||r||_2 <= tol ||b||_2.  Returns
    (x, iterations, relative residual, converged)."""
    normb = math.sqrt(float(np.vdot(b, b)))
    if normb == 0.0:
        return np.zeros_like(b), 0, 0.0, True
    x = x0.copy()
    r = b - A(x)
    normr = math.sqrt(float(np.vdot(r, r)))
    if normr <= tol * normb:
        return x, 0, normr / normb, True
    z = M(r)
    p = z.copy()
    rz = float(np.vdot(r, z))
    for k in range(1, maxit + 1):
        q = A(p)
        alpha = rz / float(np.vdot(p, q))
        x = x + alpha * p
        r = r - alpha * q
        normr = math.sqrt(float(np.vdot(r, r)))
        if normr <= tol * normb:
            return x, k, normr / normb, True
        z = M(r)
        rz_new = float(np.vdot(r, z))
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, maxit, normr / normb, False


def apply_K(d, sc, w, X):
    """The merged x-step matrix of (3.8) in the scaled variables, applied to
    X = (y, u, p): symmetric indefinite, with diagonal (1,1), (2,2) blocks."""
    y, u, p = X
    return (tcol(sc.My) * y + apply_BT(d, sc, p),
            tcol(sc.Mu) * u + sc.k_u * p,
            apply_B(d, sc, y) + sc.k_u * u - (w.delta / w.rho) * p)


def apply_Kt_inv(tab, sc, R):
    """Inverse of the block-diagonal preconditioner K~ of eq. (3.12).  The
    (1,1), (2,2) blocks M_y, M_u are diagonal and taken exactly.  The third
    block approximates the Schur complement M_p + B M_y^{-1} B^T of the p block
    (eliminating y and u from (3.8)); with the scalar blocks a, mbar_p and the
    circulant C_3(B) that is mbar_p + C_3 C_3^* / a = (mbar_p / a) S~ (or the
    matching S^ with precond_kind = 1), so its inverse is (a / mbar_p) S~^{-1}."""
    ry, ru, rp = R
    return (ry / tcol(sc.My), ru / tcol(sc.Mu), (tab["a"] / tab["mbar_p"]) * apply_precond(tab, rp))


def _bdot(X, Y):
    return float(sum(np.vdot(x, y) for x, y in zip(X, Y)))


def minres(A, M, b, x0, tol, maxit):
    """Preconditioned MINRES (Lanczos in the M^{-1} inner product, Givens QR of
    the tridiagonal) for symmetric A and symmetric positive definite M, on
    tuples of fields.  Stops when the M^{-1}-norm of the residual is at most
    tol times that of b; with tol = 0 it runs exactly maxit iterations.
    Returns (x, iterations, relative residual, converged)."""
    zb = M(b)
    nb = math.sqrt(max(_bdot(zb, b), 0.0))
    if nb == 0.0:
        return tuple(np.zeros_like(v) for v in b), 0, 0.0, True
    x = tuple(v.copy() for v in x0)
    v = tuple(bb - ax for bb, ax in zip(b, A(x)))
    z = M(v)
    g = math.sqrt(max(_bdot(z, v), 0.0))
    if g <= tol * nb:
        return x, 0, g / nb, True
    v_old = tuple(np.zeros_like(f) for f in v)
    w_old = tuple(np.zeros_like(f) for f in v)
    w_cur = tuple(np.zeros_like(f) for f in v)
    g_old = 1.0
    eta = g
    c_old = c = 1.0
    s_old = s = 0.0
    res = g
    for k in range(1, maxit + 1):
        zn = tuple(f / g for f in z)  # z_k normalised
        q = A(zn)
        dlt = _bdot(q, zn)
        # next Lanczos vector (v held unnormalised: v_k = v / g)
        v_new = tuple(qq - (dlt / g) * vv - (g / g_old) * vo for qq, vv, vo in zip(q, v, v_old))
        z_new = M(v_new)
        g_new = math.sqrt(max(_bdot(z_new, v_new), 0.0))
        # Givens rotation of the new column of the tridiagonal
        a0 = c * dlt - c_old * s * g
        a1 = math.hypot(a0, g_new)
        a2 = s * dlt + c_old * c * g
        a3 = s_old * g
        c_new, s_new = a0 / a1, g_new / a1
        w_new = tuple((zz - a3 * wo - a2 * wc) / a1 for zz, wo, wc in zip(zn, w_old, w_cur))
        x = tuple(xx + c_new * eta * ww for xx, ww in zip(x, w_new))
        eta = -s_new * eta
        res = abs(eta)
        if tol > 0 and res <= tol * nb:
            return x, k, res / nb, True
        v_old, v, z = v, v_new, z_new
        w_old, w_cur = w_cur, w_new
        g_old, g = g, g_new
        c_old, c = c, c_new
        s_old, s = s, s_new
    return x, maxit, res / nb, tol > 0 and res <= tol * nb


@dataclasses.dataclass
class AdmmResult:
    y: np.ndarray
    u: np.ndarray
    zy: np.ndarray
    zu: np.ndarray
    p: np.ndarray
    wy: np.ndarray
    wu: np.ndarray
    iters: int
    pcg_iters: list
    r_p: float
    r_y: float
    r_u: float
    converged: bool
    psi: float
    e_u: float = 1.0


def admm_solve(w, *, iters: Optional[int] = None, solver: Optional[str] = None,
               krylov_tol: Optional[float] = None, state=None) -> AdmmResult:
    """Run Algorithm 1 on workload `w` from all-zero iterates (or `state`).

    iters   -- if given, run exactly this many iterations (no stopping test)
    solver  -- "pcg" (PCG with S~, warm-started from the previous y),
               "minres" (MINRES on the merged system (3.8) with K~ of
               eq. (3.12), warm-started from the previous (y, u, p); y is
               kept and u, p recovered from it as in step 3), or
               "direct" (dense Cholesky of S; tiny grids only)
    """
    if solver is None:
        solver = "minres" if getattr(w, "krylov_solver", 0) == 1 else "pcg"
    d = op.disc_from(w)
    sc = scalars(w, d)
    tab = precond_tables(w, d)
    shape = w.shape
    yhat = np.asarray(w.yhat, dtype=np.float64)
    g = np.zeros(shape) if w.g is None else np.asarray(w.g, dtype=np.float64)
    h = sc.psi * g
    if state is None:
        y, u, zy, zu, p, wy, wu = (np.zeros(shape) for _ in range(7))
    else:
        y, u, zy, zu, p, wy, wu = (np.array(a, dtype=np.float64) for a in state)
    ktol = w.krylov_tol if krylov_tol is None else krylov_tol
    J1 = tcol(sc.wts)
    My, Mu, Mp = tcol(sc.My), tcol(sc.Mu), tcol(sc.Mp)
    rho, delta = w.rho, w.delta
    prox = bool(getattr(w, "prox", 0))
    if prox:
        Rdy, Rdu = sc.cy - J1, sc.cu - w.gamma * J1  # diagonals of R_y, R_u

    Schol = None
    if solver == "direct":
        D = op.assemble_D(d)
        Bm = sc.psi * D
        S = np.diag(np.repeat(sc.My, w.nx * w.ny)) + Bm.T @ np.diag(1.0 / np.repeat(sc.Mp, w.nx * w.ny)) @ Bm
        Schol = np.linalg.cholesky(S)

    A = lambda v: apply_S(d, sc, v)
    if getattr(w, "precond_kind", 0) == 2:
        # Delta S~^{-1} Delta: the diagonal scaling for variable coefficients
        if solver == "minres":
            raise ValueError("precond_kind 2 is a PCG preconditioner")
        delta_s = scaling_factor(diag_S(w, d, sc.My, sc.Mp, sc.psi))
        M = lambda v: apply_precond_scaled(tab, delta_s, v)
    else:
        M = lambda v: apply_precond(tab, v)
    pcg_counts = []
    maxit = w.admm_maxit if iters is None else iters
    r_p = r_y = r_u = math.inf
    converged = False
    j = 0
    for j in range(1, maxit + 1):
        # 1. right-hand sides of the merged system (3.8)
        if prox:
            # Algorithm 2: the proximal terms' share of the right-hand side, at
            # the previous iterate (y, u)
            Ry = (rho * (J1 * yhat - sc.e_y * wy + sc.e_y ** 2 * zy / delta + Rdy * y)
                  + (1 - rho) * apply_BT(d, sc, p))
            Ru = rho * (-sc.e_u * wu + sc.e_u ** 2 * zu / delta + Rdu * u) + (1 - rho) * sc.k_u * p
        else:
            Ry = rho * (J1 * yhat - sc.e_y * wy + sc.e_y ** 2 * zy / delta) + (1 - rho) * apply_BT(d, sc, p)
            Ru = rho * (-sc.e_u * wu + sc.e_u ** 2 * zu / delta) + (1 - rho) * sc.k_u * p
        r = sc.k_u * Ru / Mu - h + (delta / rho) * p
        b = Ry - apply_BT(d, sc, r / Mp)
        # 2. normal equations (3.9)
        if solver in ("pcg", "minres"):
            if getattr(w, "tol_mode", 0) == 1:
                # Sec. 6.1: 0.05 max{min of the previous iteration's three
                # residuals, 1e-4}; before the first iteration the minimum is 0
                prev = 0.0 if j == 1 else min(r_p, r_y, r_u)
                ktol = 0.05 * max(prev, 1e-4)
            cold = getattr(w, "pcg_cold_start", 0)
            if solver == "pcg":
                x0 = np.zeros(shape) if cold else y
                y, it, _, _ = pcg(A, M, b, x0, ktol, w.krylov_maxit)
            else:
                rhs = (Ry, Ru, h - (delta / rho) * p)
                X0 = tuple(np.zeros(shape) for _ in range(3)) if cold else (y, u, p)
                (y, _, _), it, _, _ = minres(lambda X: apply_K(d, sc, w, X), lambda R: apply_Kt_inv(tab, sc, R),
                                             rhs, X0, ktol, w.krylov_maxit)
            pcg_counts.append(it)
        else:
            Lc = Schol
            y = np.linalg.solve(Lc.T, np.linalg.solve(Lc, b.ravel())).reshape(shape)
            pcg_counts.append(0)
        # 3. recover p (dual update merged into the x-step) and u
        By = apply_B(d, sc, y)
        p = (By + r) / Mp
        u = (Ru - sc.k_u * p) / Mu
        # 4. z-step: projection onto the box
        zy = np.clip(y + delta * wy / sc.e_y, w.ya, w.yb)
        zu = np.clip(u + delta * wu / sc.e_u, w.ua, w.ub)
        # 5. dual updates
        wy = wy + (rho / delta) * sc.e_y * (y - zy)
        wu = wu + (rho / delta) * sc.e_u * (u - zu)
        # 6. termination test (Sec. 6.1)
        r_p = float(np.max(np.abs(By + sc.k_u * u - h)))
        r_y = float(np.max(np.abs(y - zy)))
        r_u = float(np.max(np.abs(u - zu)))
        if iters is None and max(r_p, r_y, r_u) <= w.admm_tol:
            converged = True
            break
    return AdmmResult(y=y, u=u, zy=zy, zu=zu, p=p, wy=wy, wu=wu, iters=j, pcg_iters=pcg_counts,
                      r_p=r_p, r_y=r_y, r_u=r_u, converged=converged, psi=sc.psi, e_u=sc.e_u)


def xstep_block_solve(w, yhat, zy, zu, p, wy, wu, g=None, y_prev=None, u_prev=None):
    """Reference for steps 1-3: solve the merged 3x3 block system (3.8) densely
    for (y, u, p+) in the scaled variables (tiny grids only).  With w.prox the
    system is the generalized x-step of Sec. 3.3.2: scaled-identity (1,1) and
    (2,2) blocks and the proximal terms at (y_prev, u_prev) on the right."""
    d = op.disc_from(w)
    sc = scalars(w, d)
    N = w.N
    Bm = sc.psi * op.assemble_D(d)
    J1 = np.repeat(sc.wts, w.nx * w.ny)
    J2 = w.gamma * J1
    rho, delta = w.rho, w.delta
    I = np.eye(N)
    g = np.zeros(N) if g is None else g.ravel()
    if getattr(w, "prox", 0):
        A11 = rho * (sc.cy + sc.e_y ** 2 / delta) * I
        A22 = rho * (sc.cu + sc.e_u ** 2 / delta) * I
        ex_y = rho * (sc.cy - J1) * y_prev.ravel()
        ex_u = rho * (sc.cu - J2) * u_prev.ravel()
    else:
        A11 = np.diag(rho * (J1 + sc.e_y ** 2 / delta))
        A22 = np.diag(rho * (J2 + sc.e_u ** 2 / delta))
        ex_y = ex_u = 0.0
    K = np.block([
        [A11, np.zeros((N, N)), Bm.T],
        [np.zeros((N, N)), A22, sc.k_u * I],
        [Bm, sc.k_u * I, -(delta / rho) * I],
    ])
    rhs = np.concatenate([
        rho * (J1 * yhat.ravel() - sc.e_y * wy.ravel() + sc.e_y ** 2 * zy.ravel() / delta)
        + ex_y + (1 - rho) * Bm.T @ p.ravel(),
        rho * (-sc.e_u * wu.ravel() + sc.e_u ** 2 * zu.ravel() / delta) + ex_u + (1 - rho) * sc.k_u * p.ravel(),
        sc.psi * g - (delta / rho) * p.ravel(),
    ])
    sol = np.linalg.solve(K, rhs)
    shp = w.shape
    return sol[:N].reshape(shp), sol[N:2 * N].reshape(shp), sol[2 * N:].reshape(shp)
