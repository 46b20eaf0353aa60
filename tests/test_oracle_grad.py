"""Pins for the gradients of the optimal value (envelope theorem on eq. (3.5))."""
import numpy as np
import pytest

import workloads as W
from oracle import admm, grad, kkt


def problem(**kw):
    w = W.small_mixed(nx=6, ny=5, nt=3).replace(alpha=1.4, beta=1.6, **kw)
    w.yhat = 3.0 * W.target_sinusoid_sum(6, 5, 3, W.BASE_SEED + 3)
    return w


def optimum(w):
    r = admm.admm_solve(w.replace(admm_tol=1e-9))
    pol = kkt.polish(w, r.zy, r.zu)
    assert pol["ok"]
    return r, pol


def active_set(w, pol):
    return ((pol["u"] <= w.ua + 1e-12) | (pol["u"] >= w.ub - 1e-12))


@pytest.fixture(scope="module")
def base():
    w = problem()
    r, pol = optimum(w)
    return w, r, pol


def test_adjoint_multiplier_matches_polish_and_admm(base):
    w, r, pol = base
    lam = grad.adjoint_multiplier(w, pol["y"], pol["mu_y"])
    assert kkt.rel(lam, pol["lam"]) < 1e-10
    lam_admm, _, _ = kkt.multipliers(r)
    assert kkt.rel(lam_admm, pol["lam"]) < 1e-5


def test_gradient_wrt_target_central_difference(base):
    w, r, pol = base
    gy, _, _ = grad.gradients(w, pol["y"], pol["lam"])
    rng = np.random.Generator(np.random.PCG64(9))
    h = 1e-6
    for _ in range(3):
        idx = tuple(int(rng.integers(0, s)) for s in w.shape)
        wp, wm = w.replace(yhat=w.yhat.copy()), w.replace(yhat=w.yhat.copy())
        wp.yhat[idx] += h
        wm.yhat[idx] -= h
        _, pp = optimum(wp)
        _, pm = optimum(wm)
        assert np.array_equal(active_set(w, pp), active_set(w, pol))
        fd = (pp["J"] - pm["J"]) / (2 * h)
        assert abs(fd - gy[idx]) < 1e-7 * max(1.0, abs(gy[idx]))


@pytest.mark.parametrize("which", ["alpha", "beta"])
def test_gradient_wrt_orders_central_difference(base, which):
    w, r, pol = base
    _, ga, gb = grad.gradients(w, pol["y"], pol["lam"])
    g = ga if which == "alpha" else gb
    h = 1e-6
    a0 = getattr(w, which)
    _, pp = optimum(w.replace(**{which: a0 + h}))
    _, pm = optimum(w.replace(**{which: a0 - h}))
    assert np.array_equal(active_set(w, pp), active_set(w, pol))
    fd = (pp["J"] - pm["J"]) / (2 * h)
    assert abs(fd - g) < 1e-6 * max(abs(g), 1e-3), (fd, g)


def test_adjoint_time_stepping_equals_sparse_lu(base):
    w, r, pol = base
    a = grad.adjoint_multiplier(w, pol["y"], pol["mu_y"], method="lu")
    b = grad.adjoint_multiplier(w, pol["y"], pol["mu_y"], method="steps")
    assert kkt.rel(b, a) < 1e-11
