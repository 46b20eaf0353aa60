"""Objective, KKT residuals and the active-set polish -- oracle, test infrastructure.

The discretised problem is the QP (3.3) specialised to Sec. 4:
    min 1/2 (y - yhat)^T J1 (y - yhat) + 1/2 u^T J2 u
    s.t. D y + s u = g,  ya <= y <= yb,  ua <= u <= ub,   J2 = gamma J1.
Its KKT conditions (unscaled multipliers lambda, mu_y, mu_u):
    J1 (y - yhat) + D^T lambda + mu_y = 0
    J2 u + s lambda + mu_u = 0
    D y + s u = g,   mu >= 0 where an upper bound is active, <= 0 at a lower.
From the ADMM iterates (scaled form) lambda = psi p, mu_y = e_y w_y,
mu_u = e_u w_u.  The paper reports a "dual infeasibility" without defining
it (Sec. 6.1); here it is the max-norm of the two stationarity residuals.
"""
from __future__ import annotations

import math

import numpy as np

from . import operator as op
from .admm import objective_weights, tcol


def objective(w, y, u) -> float:
    """J = 1/2 (y-yhat)^T J1 (y-yhat) + gamma/2 u^T J1 u."""
    J1 = tcol(objective_weights(w))
    e = y - w.yhat
    return 0.5 * float(np.sum(J1 * e * e)) + 0.5 * w.gamma * float(np.sum(J1 * u * u))


def el2_misfit(w, y) -> float:
    """The paper's discrete L2 misfit between state and desired state
    (Sec. 6.1): the trapezoidal rule in time (weight 1/2 on the last time
    level, the initial level being zero) and the rectangle rule in space,
    sqrt(h_x h_y h_t sum_k w_k sum_ij (y - yhat)^2)."""
    d = op.disc_from(w)
    wk = np.ones(w.nt)
    wk[-1] = 0.5
    e2 = np.sum((y - w.yhat) ** 2, axis=(1, 2))
    return float(np.sqrt(d.hx * d.hy * d.ht * np.sum(wk * e2)))


def multipliers(res):
    """Unscaled multipliers from ADMM iterates: lambda = psi p, mu_y = e_y w_y,
    mu_u = e_u w_u (e_y = 1; e_u = psi when the u copies are scaled)."""
    return res.psi * res.p, res.wy, res.e_u * res.wu


def kkt_residuals(w, y, u, lam, mu_y, mu_u, zy=None, zu=None):
    d = op.disc_from(w)
    J1 = tcol(objective_weights(w))
    g = np.zeros(w.shape) if w.g is None else w.g
    stat_y = J1 * (y - w.yhat) + op.apply_DT(d, lam) + mu_y
    stat_u = w.gamma * J1 * u + w.ctrl_sign * lam + mu_u
    prim = op.apply_D(d, y) + w.ctrl_sign * u - g
    zy = y if zy is None else zy
    zu = u if zu is None else zu
    comp_y = zy - np.clip(zy + mu_y, w.ya, w.yb)
    comp_u = zu - np.clip(zu + mu_u, w.ua, w.ub)
    return dict(
        stat_y=float(np.max(np.abs(stat_y))),
        stat_u=float(np.max(np.abs(stat_u))),
        primal=float(np.max(np.abs(prim))),
        comp_y=float(np.max(np.abs(comp_y))),
        comp_u=float(np.max(np.abs(comp_u))),
        dual_inf=float(max(np.max(np.abs(stat_y)), np.max(np.abs(stat_u)))),
    )


def bounds_flat(w):
    """(ya, yb, ua, ub) as flat arrays over the grid: scalars broadcast, and
    array-valued bounds (one value per grid point, [nt][ny][nx]) raveled."""
    return tuple(np.broadcast_to(np.asarray(b, dtype=np.float64), w.shape).ravel()
                 for b in (w.ya, w.yb, w.ua, w.ub))


def polish(w, zy, zu, tol=1e-9, method="auto"):
    """Exact optimum on the active set read off the z-iterates.

    Components of z at a finite bound are fixed there; the remaining
    equality-constrained QP's KKT system is solved with a sparse LU.  The
    result is accepted (ok=True) when it is feasible and every fixed
    component's multiplier has the sign of an optimal multiplier; KKT being
    sufficient for a convex QP, it is then the exact optimum.
    Returns dict(y, u, lam, mu_y, mu_u, ok, J).
    """
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    d = op.disc_from(w)
    N = w.N
    D = op.assemble_D_sparse(d)
    J1 = np.repeat(objective_weights(w), w.nx * w.ny)
    g = np.zeros(N) if w.g is None else w.g.ravel()
    s = w.ctrl_sign
    zy = zy.ravel()
    zu = zu.ravel()

    def active(z, lo, hi):
        lo_act = np.isfinite(lo) & (z <= lo)
        hi_act = np.isfinite(hi) & (z >= hi)
        return lo_act, hi_act

    ya, yb, ua, ub = bounds_flat(w)
    ylo, yhi = active(zy, ya, yb)
    ulo, uhi = active(zu, ua, ub)
    Ay = np.nonzero(ylo | yhi)[0]
    Au = np.nonzero(ulo | uhi)[0]
    by = np.where(ylo[Ay], ya[Ay], yb[Ay]) if len(Ay) else np.zeros(0)
    bu = np.where(ulo[Au], ua[Au], ub[Au]) if len(Au) else np.zeros(0)
    nfree = N - len(Au)
    if method == "reduced" or (method == "auto" and nfree + len(Ay) <= 1500 and w.nx * w.ny <= 4096):
        y, u, lam, my, mu = _polish_reduced(d, J1, w.gamma, s, g, w.yhat.ravel(), Au, bu, Ay, by)
        return _finish(w, y, u, lam, my, mu, ylo, yhi, ulo, uhi, tol)
    Ey = sp.csr_matrix((np.ones(len(Ay)), (np.arange(len(Ay)), Ay)), shape=(len(Ay), N))
    Eu = sp.csr_matrix((np.ones(len(Au)), (np.arange(len(Au)), Au)), shape=(len(Au), N))
    Z = lambda m, n: sp.csr_matrix((m, n))
    K = sp.bmat([
        [sp.diags(J1), Z(N, N), D.T, Ey.T, Z(N, len(Au))],
        [Z(N, N), sp.diags(w.gamma * J1), s * sp.identity(N), Z(N, len(Ay)), Eu.T],
        [D, s * sp.identity(N), Z(N, N), Z(N, len(Ay)), Z(N, len(Au))],
        [Ey, Z(len(Ay), N), Z(len(Ay), N), Z(len(Ay), len(Ay)), Z(len(Ay), len(Au))],
        [Z(len(Au), N), Eu, Z(len(Au), N), Z(len(Au), len(Ay)), Z(len(Au), len(Au))],
    ], format="csc")
    rhs = np.concatenate([J1 * w.yhat.ravel(), np.zeros(N), g, by, bu])
    sol = spla.spsolve(K, rhs)
    y = sol[:N]
    u = sol[N:2 * N]
    lam = sol[2 * N:3 * N]
    my = np.zeros(N)
    mu = np.zeros(N)
    my[Ay] = sol[3 * N:3 * N + len(Ay)]
    mu[Au] = sol[3 * N + len(Ay):]
    return _finish(w, y, u, lam, my, mu, ylo, yhi, ulo, uhi, tol)


def _polish_reduced(d, J1, gamma, s, g, yhat, Au, bu, Ay, by):
    """The same equality-constrained QP with y = D^{-1}(g - s u) eliminated:
    unknowns are the free controls u_F and the multipliers nu of the fixed
    states; D is solved directly by time stepping (op.DSolver)."""
    N = d.nx * d.ny * d.nt
    lu = op.DSolver(d)
    F = np.setdiff1d(np.arange(N), Au)
    uA = np.zeros(N)
    uA[Au] = bu
    c = lu.solve(g - s * uA)  # y for u_F = 0
    EF = np.zeros((N, len(F)))
    EF[F, np.arange(len(F))] = 1.0
    K = -s * lu.solve(EF)  # K = -s D^{-1} E_F^T
    H = K.T @ (J1[:, None] * K) + np.diag(gamma * J1[F])
    rhs1 = -K.T @ (J1 * (c - yhat))
    if len(Ay):
        KA = K[Ay, :]
        M = np.block([[H, KA.T], [KA, np.zeros((len(Ay), len(Ay)))]])
        sol = np.linalg.solve(M, np.concatenate([rhs1, by - c[Ay]]))
        uF, nu = sol[:len(F)], sol[len(F):]
    else:
        uF, nu = np.linalg.solve(H, rhs1), np.zeros(0)
    u = uA.copy()
    u[F] = uF
    y = c + K @ uF
    my = np.zeros(N)
    my[Ay] = nu
    lam = -lu.solve(J1 * (y - yhat) + my, trans=True)
    mu = np.zeros(N)
    mu[Au] = -(gamma * J1[Au] * u[Au] + s * lam[Au])
    return y, u, lam, my, mu


def _finish(w, y, u, lam, my, mu, ylo, yhi, ulo, uhi, tol):
    ya, yb, ua, ub = bounds_flat(w)
    feas = (np.all(y >= ya - tol) and np.all(y <= yb + tol)
            and np.all(u >= ua - tol) and np.all(u <= ub + tol))
    signs = (np.all(my[ylo] <= tol) and np.all(my[yhi] >= -tol)
             and np.all(mu[ulo] <= tol) and np.all(mu[uhi] >= -tol))
    shp = w.shape
    out = dict(y=y.reshape(shp), u=u.reshape(shp), lam=lam.reshape(shp), mu_y=my.reshape(shp),
               mu_u=mu.reshape(shp), ok=bool(feas and signs))
    out["J"] = objective(w, out["y"], out["u"])
    return out


def rel(a, b) -> float:
    """Relative 2-norm difference |a - b| / |b| (|a| when b = 0)."""
    nb = math.sqrt(float(np.vdot(b, b)))
    na = math.sqrt(float(np.vdot(a - b, a - b)))
    return na / nb if nb > 0 else na
