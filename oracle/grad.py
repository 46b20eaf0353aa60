"""Gradients of the optimal value J*(yhat, alpha, beta) -- oracle, test infrastructure.

By the envelope theorem applied to the Lagrangian of the QP (the unscaled form
of eq. (3.5) at a KKT point): the bounds do not depend on the data, so
    dJ*/dyhat  = -J1 (y* - yhat)
    dJ*/dalpha = lambda^T (dD/dalpha) y*,   dJ*/dbeta = lambda^T (dD/dbeta) y*,
with lambda the multiplier of D y + s u = g.  D = C_t (x) I - I (x)(L_x (+) L_y)
(eq. (4.9)) gives dD/dalpha = -dL_x/dalpha, where for
L_x = c_a h^-a (diag(d+) G_a + diag(d-) G_a^T):
    dL_x/da = ((pi/2) tan(a pi/2) - ln h) L_x + c_a h^-a (diag(d+) G'_a + diag(d-) G'_a^T),
G'_a being the shifted Grünwald matrix built from the derivative weights.
The same holds along y with beta.
"""
from __future__ import annotations

import math

import numpy as np

from . import operator as op
from .admm import objective_weights, tcol
from .grunwald import riesz_factor, weight_derivatives


def dLx_dalpha(d: op.Disc, v):
    """(dL_x/dalpha) v along every x-line (dense 1-D factors)."""
    a, h, n = d.alpha, d.hx, d.nx
    G = op.shifted_grunwald(a, n)
    Gd = op.shifted_grunwald(a, n, weight_derivatives(a, n))
    c = riesz_factor(a) / h ** a
    Lv = c * (d.dplus * (v @ G.T) + d.dminus * (v @ G))
    Ldv = c * (d.dplus * (v @ Gd.T) + d.dminus * (v @ Gd))
    return ((math.pi / 2) * math.tan(a * math.pi / 2) - math.log(h)) * Lv + Ldv


def dLy_dbeta(d: op.Disc, v):
    a, h, n = d.beta, d.hy, d.ny
    G = op.shifted_grunwald(a, n)
    Gd = op.shifted_grunwald(a, n, weight_derivatives(a, n))
    c = riesz_factor(a) / h ** a
    Lv = c * (d.dplus * np.matmul(G, v) + d.dminus * np.matmul(G.T, v))
    Ldv = c * (d.dplus * np.matmul(Gd, v) + d.dminus * np.matmul(Gd.T, v))
    return ((math.pi / 2) * math.tan(a * math.pi / 2) - math.log(h)) * Lv + Ldv


def gradients(w, y, lam):
    """(dJ/dyhat, dJ/dalpha, dJ/dbeta) at the optimum (y*, lambda)."""
    d = op.disc_from(w)
    J1 = tcol(objective_weights(w))
    dyhat = -J1 * (y - w.yhat)
    dalpha = float(np.vdot(lam, -dLx_dalpha(d, y)))
    dbeta = float(np.vdot(lam, -dLy_dbeta(d, y)))
    return dyhat, dalpha, dbeta


def adjoint_multiplier(w, y, mu_y, method="lu"):
    """lambda from the adjoint (transposed) state equation
    D^T lambda = -J1 (y - yhat) - mu_y: sparse LU of D^T ("lu"), or backward
    time stepping with a dense LU of the 2-D block ("steps"); small grids."""
    d = op.disc_from(w)
    J1 = tcol(objective_weights(w))
    rhs = (-J1 * (y - w.yhat) - mu_y).ravel()
    if method == "steps":
        return op.DSolver(d).solve(rhs, trans=True).reshape(w.shape)
    import scipy.sparse.linalg as spla

    D = op.assemble_D_sparse(d)
    return spla.spsolve(D.T.tocsc(), rhs).reshape(w.shape)
