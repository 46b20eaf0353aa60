"""Pins for Algorithm 1 with the merged x-step (Sec. 3.1) and the KKT polish."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import admm, kkt
from oracle import operator as op
from oracle import precond as pc


def tiny(**kw):
    w = W.small(nx=5, ny=4, nt=3).replace(**kw)
    w.dplus = W.coef_sine_x(5, 4)
    return w


def random_state(w, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.standard_normal(w.shape) for _ in range(5)]


@pytest.mark.parametrize("ctrl_sign", [1.0, -1.0])
@pytest.mark.parametrize("obj_weights", [0, 1])
@pytest.mark.parametrize("rho,delta", [(1.0, 1.0), (1.618, 0.4)])
def test_reduced_xstep_equals_block_solve(ctrl_sign, obj_weights, rho, delta):
    """Steps 1-3 (elimination + normal equations) reproduce the 3x3 merged
    system (3.8) solved densely; this fixes the sign of the M_u^{-1} term."""
    w = tiny(ctrl_sign=ctrl_sign, obj_weights=obj_weights, rho=rho, delta=delta)
    zy, zu, p, wy, wu = random_state(w, 7)
    y_ref, u_ref, p_ref = admm.xstep_block_solve(w, w.yhat, zy, zu, p, wy, wu)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    J1, Mu, Mp = admm.tcol(sc.wts), admm.tcol(sc.Mu), admm.tcol(sc.Mp)
    Ry = rho * (J1 * w.yhat - sc.e_y * wy + sc.e_y ** 2 * zy / delta) + (1 - rho) * admm.apply_BT(d, sc, p)
    Ru = rho * (-sc.e_u * wu + sc.e_u ** 2 * zu / delta) + (1 - rho) * sc.k_u * p
    r = sc.k_u * Ru / Mu + (delta / rho) * p  # g = 0
    b = Ry - admm.apply_BT(d, sc, r / Mp)
    Bm = sc.psi * op.assemble_D(d)
    S = np.diag(np.repeat(sc.My, w.nx * w.ny)) + Bm.T @ np.diag(1 / np.repeat(sc.Mp, w.nx * w.ny)) @ Bm
    y = np.linalg.solve(S, b.ravel()).reshape(w.shape)
    pp = (admm.apply_B(d, sc, y) + r) / Mp
    u = (Ru - sc.k_u * pp) / Mu
    assert kkt.rel(y, y_ref) < 1e-12
    assert kkt.rel(u, u_ref) < 1e-12
    assert kkt.rel(pp, p_ref) < 1e-12
    # the printed minus sign does not reproduce the block solve
    r_bad = -sc.k_u * Ru / Mu + (delta / rho) * p
    b_bad = Ry - admm.apply_BT(d, sc, r_bad / Mp)
    y_bad = np.linalg.solve(S, b_bad.ravel()).reshape(w.shape)
    assert kkt.rel(y_bad, y_ref) > 1e-3


def test_normal_matrix_is_spd_with_lower_bound():
    w = tiny(rho=1.3, delta=0.5)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    Bm = sc.psi * op.assemble_D(d)
    S = np.diag(np.repeat(sc.My, w.nx * w.ny)) + Bm.T @ np.diag(1 / np.repeat(sc.Mp, w.nx * w.ny)) @ Bm
    np.testing.assert_allclose(S, S.T, atol=1e-12)
    ev = np.linalg.eigvalsh(S)
    assert ev.min() >= w.rho / w.delta - 1e-12  # Thm 3.1 proof: S >= rho/delta I (J1 >= 0)
    # the line-wise operator agrees with the dense matrix
    v = W.random_field(w.shape, 1)
    np.testing.assert_allclose(admm.apply_S(d, sc, v).ravel(), S @ v.ravel(), rtol=1e-12)


def test_pcg_solves_normal_equations():
    w = W.small(nx=8, ny=8, nt=4)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    tab = pc.precond_tables(w, d)
    b = W.random_field(w.shape, 2)
    x, it, relres, ok = admm.pcg(lambda v: admm.apply_S(d, sc, v), lambda v: pc.apply_precond(tab, v),
                                 b, np.zeros(w.shape), 1e-12, 500)
    assert ok and 0 < it < 100
    Bm = sc.psi * op.assemble_D(d)
    S = np.diag(np.repeat(sc.My, w.nx * w.ny)) + Bm.T @ np.diag(1 / np.repeat(sc.Mp, w.nx * w.ny)) @ Bm
    xs = np.linalg.solve(S, b.ravel())
    assert kkt.rel(x.ravel(), xs) < 1e-10
    # the circulant preconditioner keeps the count far below the unpreconditioned one
    _, it_plain, _, _ = admm.pcg(lambda v: admm.apply_S(d, sc, v), lambda v: v, b, np.zeros(w.shape),
                                 1e-12, 5000)
    assert it < it_plain


def test_pcg_zero_rhs_and_warm_start():
    w = W.small(nx=4, ny=4, nt=2)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    A = lambda v: admm.apply_S(d, sc, v)
    x, it, _, ok = admm.pcg(A, lambda v: v, np.zeros(w.shape), np.ones(w.shape), 1e-10, 10)
    assert it == 0 and ok and np.all(x == 0)
    b = W.random_field(w.shape, 3)
    xs, _, _, _ = admm.pcg(A, lambda v: v, b, np.zeros(w.shape), 1e-14, 500)
    x, it, _, ok = admm.pcg(A, lambda v: v, b, xs, 1e-10, 10)
    assert it == 0 and ok


@pytest.fixture(scope="module")
def small_result():
    w = W.small()
    return w, admm.admm_solve(w)


def test_small_case_saturates_at_lower_bound(small_result):
    """The 16^2 x 8 case: every control sits at u = -1 and y* = D^{-1} 1."""
    w, r = small_result
    assert r.converged and 1000 < r.iters < 2500
    pol = kkt.polish(w, r.zy, r.zu)
    assert pol["ok"]
    d = op.disc_from(w)
    y1 = np.linalg.solve(op.assemble_D(d), np.ones(w.N)).reshape(w.shape)
    assert kkt.rel(pol["y"], y1) < 1e-13
    assert np.max(np.abs(pol["u"] + 1.0)) < 1e-12
    # the ADMM iterate is within the tolerance's reach of the exact optimum
    assert np.max(np.abs(r.y - pol["y"])) < 1e-5
    assert np.max(np.abs(r.zu + 1.0)) == 0.0
    res = kkt.kkt_residuals(w, r.y, r.u, *kkt.multipliers(r), r.zy, r.zu)
    assert res["primal"] < 1e-5 and res["dual_inf"] < 1e-5


def test_mixed_active_box_matches_bounded_least_squares():
    """Control-only box: the QP is a bounded least-squares problem in u with
    y = D^{-1}(g - s u); scipy's lsq_linear is an independent solver."""
    from scipy.optimize import lsq_linear

    w = W.small_mixed(nx=8, ny=8, nt=4)
    r = admm.admm_solve(w)
    assert r.converged
    pol = kkt.polish(w, r.zy, r.zu)
    assert pol["ok"]
    d = op.disc_from(w)
    Dinv = np.linalg.inv(op.assemble_D(d))
    A = np.vstack([-w.ctrl_sign * Dinv, math.sqrt(w.gamma) * np.eye(w.N)])
    b = np.concatenate([w.yhat.ravel(), np.zeros(w.N)])
    ls = lsq_linear(A, b, bounds=(w.ua, w.ub), method="bvls", tol=1e-14)
    nact = int(np.sum((ls.x <= w.ua + 1e-12) | (ls.x >= w.ub - 1e-12)))
    assert 0 < nact < w.N  # genuinely mixed
    np.testing.assert_allclose(pol["u"].ravel(), ls.x, atol=1e-9)
    assert np.max(np.abs(r.u.ravel() - ls.x)) < 1e-4


def test_state_bound_active_kkt():
    w = W.small_state(nx=8, ny=8, nt=4)
    r = admm.admm_solve(w)
    assert r.converged
    pol = kkt.polish(w, r.zy, r.zu)
    assert pol["ok"]
    assert np.sum(r.zy >= w.yb) > 0
    res = kkt.kkt_residuals(w, pol["y"], pol["u"], pol["lam"], pol["mu_y"], pol["mu_u"])
    assert max(res.values()) < 1e-8
    assert np.max(np.abs(r.y - pol["y"])) < 1e-4


def test_inactive_box_is_equality_constrained_solution():
    w = W.small(nx=6, ny=6, nt=4, ua=-1e6, ub=1e6)
    r = admm.admm_solve(w)
    pol = kkt.polish(w, r.zy, r.zu)
    assert pol["ok"] and r.converged
    # equality-constrained optimum from the normal equations of the reduced LSQ
    d = op.disc_from(w)
    Dinv = np.linalg.inv(op.assemble_D(d))
    K = -w.ctrl_sign * Dinv
    u = np.linalg.solve(K.T @ K + w.gamma * np.eye(w.N), K.T @ w.yhat.ravel())
    np.testing.assert_allclose(pol["u"].ravel(), u, rtol=1e-8, atol=1e-10)


def test_headline_shape_with_control_as_sink_is_zero():
    """With D y + u = g, g = 0, u >= 0 and D an M-matrix, y <= 0 <= yhat; the
    optimum is y = u = 0 exactly."""
    w = W.headline(nx=8, ny=8, nt=4, ctrl_sign=1.0)
    r = admm.admm_solve(w)
    pol = kkt.polish(w, r.zy, r.zu)
    assert pol["ok"]
    assert np.max(np.abs(pol["y"])) < 1e-14 and np.max(np.abs(pol["u"])) < 1e-14
    assert np.max(np.abs(r.y)) < 1e-5


def test_pcg_and_direct_inner_solves_agree():
    w = W.small_mixed(nx=6, ny=6, nt=3)
    a = admm.admm_solve(w, iters=40, krylov_tol=1e-13)
    b = admm.admm_solve(w, iters=40, solver="direct")
    assert kkt.rel(a.y, b.y) < 1e-10 and kkt.rel(a.u, b.u) < 1e-10


def test_trapezoidal_weights_and_rho_option():
    w = W.small_mixed(nx=6, ny=6, nt=4, obj_weights=1, rho=1.618, delta=0.4, admm_tol=1e-8)
    r = admm.admm_solve(w)
    assert r.converged
    pol = kkt.polish(w, r.zy, r.zu)
    assert pol["ok"]
    # u = (g - D y)/s amplifies the y error by |D| ~ h^-alpha; compare y tightly
    assert np.max(np.abs(r.y - pol["y"])) < 1e-5
    assert kkt.rel(r.u, pol["u"]) < 1e-4


@pytest.mark.parametrize("kind", ["mixed", "state"])
def test_reduced_polish_equals_full_kkt_polish(kind):
    """The reduced active-set polish (y eliminated through a sparse LU of D)
    solves the same KKT system as the full sparse saddle-point solve."""
    w = (W.small_mixed if kind == "mixed" else W.small_state)(nx=8, ny=6, nt=4)
    r = admm.admm_solve(w)
    a = kkt.polish(w, r.zy, r.zu, method="full")
    b = kkt.polish(w, r.zy, r.zu, method="reduced")
    assert a["ok"] and b["ok"]
    for k in ("y", "u", "lam", "mu_y", "mu_u"):
        assert np.max(np.abs(a[k] - b[k])) <= 1e-9 * max(1.0, np.max(np.abs(a[k]))), k
    assert abs(a["J"] - b["J"]) <= 1e-12 * abs(a["J"])
