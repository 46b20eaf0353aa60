"""Pins for Algorithm 2, the generalized (proximal) ADMM of Sec. 3.3.2, with
R_y = c_y I - J1 and R_u = c_u I - J2: the x-step against the printed
coefficient matrix solved densely, the reduction to Algorithm 1 when R = 0,
the KKT optimum as a fixed point, and convergence to the same optimum as
Algorithm 1."""
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


def rand_fields(w, seed, count):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.standard_normal(w.shape) for _ in range(count)]


@pytest.mark.parametrize("obj_weights", [0, 1])
@pytest.mark.parametrize("cy,cu,rho,delta", [(0.0, 0.0, 1.0, 1.0), (1.7, 3e-3, 0.8, 0.4)])
def test_generalized_xstep_equals_block_solve(obj_weights, cy, cu, rho, delta):
    """One iteration from a random state (inner solve direct): y, u, p equal
    the dense solve of the generalized x-step's block system (scaled-identity
    (1,1) and (2,2) blocks, proximal terms at the previous y and u)."""
    w = tiny(prox=1, prox_cy=cy, prox_cu=cu, obj_weights=obj_weights, rho=rho, delta=delta, ctrl_sign=-1.0)
    y0, u0, zy, zu, p, wy, wu = rand_fields(w, 11, 7)
    r = admm.admm_solve(w, iters=1, solver="direct", state=(y0, u0, zy, zu, p, wy, wu))
    y, u, pp = admm.xstep_block_solve(w, w.yhat, zy, zu, p, wy, wu, y_prev=y0, u_prev=u0)
    assert kkt.rel(r.y, y) < 1e-11 and kkt.rel(r.u, u) < 1e-11 and kkt.rel(r.p, pp) < 1e-11
    # the previous iterate matters (R != 0 somewhere), with the sign printed
    if obj_weights == 1 or cy > 0:
        yb, _, _ = admm.xstep_block_solve(w, w.yhat, zy, zu, p, wy, wu, y_prev=-y0, u_prev=-u0)
        assert kkt.rel(yb, y) > 1e-6


def test_scaled_identity_blocks():
    w = tiny(prox=1, prox_cy=2.5, prox_cu=0.01, obj_weights=1, rho=0.9, delta=0.3)
    sc = admm.scalars(w, op.disc_from(w))
    assert sc.cy == 2.5 and sc.cu == 0.01
    np.testing.assert_array_equal(sc.My, np.full(w.nt, 0.9 * (2.5 + 1 / 0.3)))
    np.testing.assert_array_equal(sc.Mu, np.full(w.nt, 0.9 * (0.01 + sc.e_u ** 2 / 0.3)))
    # the preconditioner's scalars are then exact: a = M_y, mbar_p = M_p
    tab = pc.precond_tables(w, op.disc_from(w))
    assert tab["a"] == sc.My[0] and abs(tab["mbar_p"] - sc.Mp[0]) <= 1e-15 * sc.Mp[0]
    # defaults: the smallest admissible constants
    w0 = w.replace(prox_cy=0.0, prox_cu=0.0)
    s0 = admm.scalars(w0, op.disc_from(w0))
    assert s0.cy == 1.0 and s0.cu == w.gamma


def test_zero_proximal_term_is_algorithm_1():
    """J1 = I, c_y = 1, c_u = gamma: R = 0 and Algorithm 2 is Algorithm 1."""
    w = W.small_mixed(nx=8, ny=6, nt=4)
    a = admm.admm_solve(w, iters=25)
    b = admm.admm_solve(w.replace(prox=1), iters=25)
    assert a.pcg_iters == b.pcg_iters
    for k in ("y", "u", "zy", "zu", "p", "wy", "wu"):
        np.testing.assert_allclose(getattr(b, k), getattr(a, k), rtol=0, atol=1e-13 * max(1, np.abs(getattr(a, k)).max()))


def kkt_state(w, pol, sc):
    """ADMM state (scaled multipliers) of an exact KKT point."""
    return (pol["y"], pol["u"], pol["y"].copy(), pol["u"].copy(), pol["lam"] / sc.psi, pol["mu_y"] / sc.e_y,
            pol["mu_u"] / sc.e_u)


@pytest.mark.parametrize("kind", ["mixed", "state"])
def test_kkt_point_is_a_fixed_point(kind):
    """From the exact optimum (active-set polish of an Algorithm 1 run) one
    Algorithm 2 iteration returns the same point; R_y, R_u are nonzero."""
    w = (W.small_mixed if kind == "mixed" else W.small_state)(nx=6, ny=5, nt=4, obj_weights=1)
    r = admm.admm_solve(w)
    pol = kkt.polish(w, r.zy, r.zu)
    assert r.converged and pol["ok"]
    w2 = w.replace(prox=1, prox_cy=1.5, prox_cu=5 * w.gamma, rho=0.9)
    sc = admm.scalars(w2, op.disc_from(w2))
    st = kkt_state(w, pol, sc)
    out = admm.admm_solve(w2, iters=1, solver="direct", state=st)
    for k, ref in zip(("y", "u", "zy", "zu", "p", "wy", "wu"), st):
        got = getattr(out, k)
        assert np.max(np.abs(got - ref)) <= 1e-8 * max(1.0, np.max(np.abs(ref))), k


@pytest.mark.parametrize("kind,cy,cu_factor", [("mixed", 0.0, 0.0), ("state", 2.0, 10.0), ("mixed", 1.2, 3.0)])
def test_converges_to_the_algorithm_1_optimum(kind, cy, cu_factor):
    w = (W.small_mixed if kind == "mixed" else W.small_state)(nx=8, ny=8, nt=4, obj_weights=1)
    ref = kkt.polish(w, *(lambda r: (r.zy, r.zu))(admm.admm_solve(w)))
    assert ref["ok"]
    w2 = w.replace(prox=1, prox_cy=cy, prox_cu=cu_factor * w.gamma, rho=1.0, admm_tol=1e-8)
    r = admm.admm_solve(w2)
    assert r.converged
    pol = kkt.polish(w2, r.zy, r.zu)
    assert pol["ok"]
    assert np.max(np.abs(pol["y"] - ref["y"])) <= 1e-9 and np.max(np.abs(pol["u"] - ref["u"])) <= 1e-7
    assert np.max(np.abs(r.y - ref["y"])) < 1e-6
