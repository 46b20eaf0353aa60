"""Pins for array-valued box bounds (one bound per grid point) in the oracle:
constant arrays reproduce the scalar-bound iterates exactly, and varying
bounds reach the optimum that scipy's bounded least squares and the KKT
conditions fix."""
import math

import numpy as np

import workloads as W
from oracle import admm, kkt
from oracle import operator as op


def grid(w):
    t = (np.arange(1, w.nt + 1) * (w.T / w.nt))[:, None, None]
    y = (np.arange(1, w.ny + 1) / (w.ny + 1))[None, :, None]
    x = (np.arange(1, w.nx + 1) / (w.nx + 1))[None, None, :]
    return t, y, x


def test_constant_arrays_equal_scalar_bounds():
    w = W.small_state(nx=8, ny=6, nt=4)
    a = admm.admm_solve(w, iters=40)
    full = lambda v: np.full(w.shape, v)
    b = admm.admm_solve(w.replace(ya=full(w.ya), yb=full(w.yb), ua=full(w.ua), ub=full(w.ub)), iters=40)
    for k in ("y", "u", "zy", "zu", "p", "wy", "wu"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k


def test_varying_control_bounds_match_bounded_least_squares():
    """Control-only box with per-point bounds: the QP is bounded least squares
    in u with y = D^{-1}(g - s u); scipy's lsq_linear takes array bounds."""
    from scipy.optimize import lsq_linear

    w = W.small(nx=8, ny=8, nt=4)
    t, y, x = grid(w)
    ua = -0.2 - 0.5 * x * np.ones(w.shape)
    ub = 0.1 + 0.8 * t * y * np.ones(w.shape)
    ua[0, :, :2] = -np.inf  # some points free below
    w = w.replace(ua=ua, ub=ub, admm_tol=1e-9)
    r = admm.admm_solve(w)
    assert r.converged
    pol = kkt.polish(w, r.zy, r.zu)
    assert pol["ok"]
    d = op.disc_from(w)
    Dinv = np.linalg.inv(op.assemble_D(d))
    A = np.vstack([-w.ctrl_sign * Dinv, math.sqrt(w.gamma) * np.eye(w.N)])
    b = np.concatenate([w.yhat.ravel(), np.zeros(w.N)])
    ls = lsq_linear(A, b, bounds=(ua.ravel(), ub.ravel()), method="bvls", tol=1e-14)
    at_lo = np.sum(ls.x <= ua.ravel() + 1e-12)
    at_hi = np.sum(ls.x >= ub.ravel() - 1e-12)
    assert at_lo > 0 and at_lo + at_hi < w.N  # genuinely mixed
    np.testing.assert_allclose(pol["u"].ravel(), ls.x, atol=1e-9)
    assert np.max(np.abs(r.u.ravel() - ls.x)) < 1e-5


def test_varying_state_bound_kkt():
    w = W.small_state(nx=8, ny=8, nt=4)
    t, y, x = grid(w)
    yb = 0.02 + 0.15 * t * (1.0 + x) * np.ones(w.shape)
    w = w.replace(yb=yb)
    r = admm.admm_solve(w)
    assert r.converged
    pol = kkt.polish(w, r.zy, r.zu)
    assert pol["ok"]
    assert np.sum(pol["y"] >= yb - 1e-12) > 0  # the varying bound is active somewhere
    assert np.all(pol["y"] <= yb + 1e-10)
    res = kkt.kkt_residuals(w, pol["y"], pol["u"], pol["lam"], pol["mu_y"], pol["mu_u"])
    assert max(res.values()) < 1e-8
    assert np.max(np.abs(r.y - pol["y"])) < 1e-4
