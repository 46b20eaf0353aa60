"""Pins for the Grünwald weights (Sec. 4, recurrence under eq. (4.4); Prop. 4.1)."""
import math

import numpy as np
import pytest
from scipy import special

from oracle.grunwald import riesz_factor, riesz_factor_derivative, weight_derivatives, weights

ORDERS = [0.3, 0.7, 1.1, 1.3, 1.5, 1.7, 1.9]


@pytest.mark.parametrize("a", ORDERS)
def test_recurrence_matches_gamma_closed_form(a):
    # g_k = Gamma(k - a) / (Gamma(-a) Gamma(k + 1)) = (-1)^k binom(a, k)
    n = 60
    g = weights(a, n)
    k = np.arange(n + 1)
    closed = (-1.0) ** k * special.binom(a, k)
    np.testing.assert_allclose(g, closed, rtol=1e-12, atol=1e-300)
    # the Gamma form itself (sign-aware log-gamma) for the non-trivial terms
    lg = special.gammaln(k[1:] - a) - special.gammaln(-a) - special.gammaln(k[1:] + 1.0)
    sgn = np.sign(special.gamma(k[1:] - a)) * np.sign(special.gamma(-a))
    np.testing.assert_allclose(g[1:], sgn * np.exp(lg), rtol=1e-11)


@pytest.mark.parametrize("a", ORDERS)
def test_partial_sums(a):
    # sum_{k<=n} g_k = (-1)^n binom(a - 1, n)
    n = 200
    g = weights(a, n)
    ps = np.cumsum(g)
    k = np.arange(n + 1)
    np.testing.assert_allclose(ps, (-1.0) ** k * special.binom(a - 1, k), rtol=1e-10, atol=1e-15)


@pytest.mark.parametrize("a", [1.1, 1.3, 1.5, 1.7, 1.9])
def test_prop41_space_orders(a):
    g = weights(a, 400)
    assert g[0] == 1.0
    assert abs(g[1] + a) < 1e-15
    assert np.all(np.diff(g[2:]) < 0) and np.all(g[2:] > 0)
    assert np.all(np.cumsum(g)[1:] < 0)
    # sum to infinity is 0: the tail decays like k^(-a-1)
    assert abs(np.sum(weights(a, 200000))) < 1e-3


@pytest.mark.parametrize("a", [0.1, 0.5, 0.9])
def test_prop41_time_orders(a):
    g = weights(a, 300)
    assert g[0] > 0 and np.all(g[1:] < 0)
    assert np.all(np.cumsum(g) > 0)


def test_integer_orders():
    np.testing.assert_array_equal(weights(1.0, 5), [1, -1, 0, 0, 0, 0])
    np.testing.assert_array_equal(weights(2.0, 5), [1, -2, 1, 0, 0, 0])


@pytest.mark.parametrize("a", [0.7, 1.2, 1.4, 1.6, 1.85])
def test_derivative_weights(a):
    n = 50
    dg = weight_derivatives(a, n)
    g = weights(a, n)
    k = np.arange(1, n + 1)
    # closed form: d/da log|g_k| = psi0(-a) - psi0(k - a)
    np.testing.assert_allclose(dg[1:], g[1:] * (special.digamma(-a) - special.digamma(k - a)),
                               rtol=1e-11, atol=1e-15)
    assert dg[0] == 0.0
    h = 1e-6
    fd = (weights(a + h, n) - weights(a - h, n)) / (2 * h)
    np.testing.assert_allclose(dg, fd, rtol=1e-7, atol=1e-10)


@pytest.mark.parametrize("a", [1.1, 1.5, 1.9])
def test_riesz_factor(a):
    c = riesz_factor(a)
    assert c > 0  # cos(a pi/2) < 0 for a in (1, 2)
    h = 1e-6
    fd = (riesz_factor(a + h) - riesz_factor(a - h)) / (2 * h)
    assert abs(riesz_factor_derivative(a) - fd) < 1e-7 * abs(fd)
    assert abs(riesz_factor(2.0) - 0.5) < 1e-15
