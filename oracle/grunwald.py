"""Fractional binomial (Grünwald-Letnikov) weights -- oracle, test infrastructure.

Sec. 4, the weights under eq. (4.4): g_0 = 1 and g_k = (1 - (a+1)/k) g_{k-1},
equivalently g_k = Gamma(k-a) / (Gamma(-a) Gamma(k+1)).  The Riesz factor of
eq. (4.1)/(4.7) is -1 / (2 cos(a pi / 2)).
"""
from __future__ import annotations

import math

import numpy as np


def weights(a: float, n: int) -> np.ndarray:
    """g_0 .. g_n for order a, by the recurrence of Sec. 4 (under eq. (4.4))."""
    g = np.empty(n + 1, dtype=np.float64)
    g[0] = 1.0
    for k in range(1, n + 1):
        g[k] = (1.0 - (a + 1.0) / k) * g[k - 1]
    return g


def weight_derivatives(a: float, n: int) -> np.ndarray:
    """d g_k / d a for k = 0..n, from differentiating the recurrence in a:
    g'_0 = 0,  g'_k = (1 - (a+1)/k) g'_{k-1} - g_{k-1} / k."""
    g = weights(a, n)
    dg = np.empty(n + 1, dtype=np.float64)
    dg[0] = 0.0
    for k in range(1, n + 1):
        dg[k] = (1.0 - (a + 1.0) / k) * dg[k - 1] - g[k - 1] / k
    return dg


def riesz_factor(a: float) -> float:
    """c_a = -1 / (2 cos(a pi / 2)), eq. (4.1) and (4.7)."""
    return -1.0 / (2.0 * math.cos(a * math.pi / 2.0))


def riesz_factor_derivative(a: float) -> float:
    """d c_a / d a = c_a * (pi/2) tan(a pi / 2)."""
    return riesz_factor(a) * (math.pi / 2.0) * math.tan(a * math.pi / 2.0)
