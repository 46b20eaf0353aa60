"""Pins for the constraint matrix D (Sec. 4, eqs. (4.5)-(4.9))."""
import math

import numpy as np
import pytest
from scipy import special

import workloads as W
from oracle import operator as op
from oracle.grunwald import riesz_factor


def tiny(nx=7, ny=5, nt=4, alpha=1.3, beta=1.7, var=True):
    w = W.small(nx=nx, ny=ny, nt=nt).replace(alpha=alpha, beta=beta)
    if var:
        w.dplus = W.coef_sine_x(nx, ny)
        rng = np.random.Generator(np.random.PCG64(3))
        w.dminus = 1.0 + 0.3 * rng.uniform(size=(ny, nx))
    return w


def test_shifted_grunwald_band_structure():
    # eq. (4.6): first row (g1, g0, 0, ...), sub-diagonals g2, g3, ...
    from oracle.grunwald import weights
    n, a = 6, 1.4
    G = op.shifted_grunwald(a, n)
    g = weights(a, n)
    assert G[0, 0] == g[1] and G[0, 1] == g[0] and np.all(G[0, 2:] == 0)
    assert G[n - 1, 0] == g[n]
    assert np.all(np.triu(G, 2) == 0)


def _rl_left_poly(coefs, a, x):
    """Left Riemann-Liouville derivative from 0 of sum_p c_p x^p."""
    return sum(c * special.gamma(p + 1) / special.gamma(p + 1 - a) * x ** (p - a)
               for p, c in coefs.items())


@pytest.mark.parametrize("a", [1.3, 1.5, 1.8])
def test_riesz_matrix_approximates_riesz_derivative(a):
    # f(x) = x^2 (1-x)^2 on (0,1): left RL derivative in closed form; the
    # right-sided one is the left one reflected (f is symmetric about 1/2).
    coefs = {2: 1.0, 3: -2.0, 4: 1.0}
    errs = []
    for n in (200, 400, 800):
        h = 1.0 / (n + 1)
        x = h * np.arange(1, n + 1)
        f = x ** 2 * (1 - x) ** 2
        L = op.line_matrix(a, h, n, np.ones(n), np.ones(n))
        exact = riesz_factor(a) * (_rl_left_poly(coefs, a, x) + _rl_left_poly(coefs, a, 1 - x))
        mid = (x > 0.25) & (x < 0.75)  # away from the boundary layers
        errs.append(np.max(np.abs(L @ f - exact)[mid]))
    # first-order scheme: the interior error halves with h
    assert 0.45 < errs[1] / errs[0] < 0.55 and 0.45 < errs[2] / errs[1] < 0.55
    assert errs[2] < 0.01 * np.max(np.abs(exact))


def test_order_two_is_five_point_heat_operator():
    nx, ny, nt = 6, 5, 3
    w = W.small(nx=nx, ny=ny, nt=nt).replace(alpha=2.0, beta=2.0)
    d = op.disc_from(w)
    D = op.assemble_D(d)
    Tx = (np.eye(nx, k=1) - 2 * np.eye(nx) + np.eye(nx, k=-1)) / d.hx ** 2
    Ty = (np.eye(ny, k=1) - 2 * np.eye(ny) + np.eye(ny, k=-1)) / d.hy ** 2
    lap = np.kron(np.eye(ny), Tx) + np.kron(Ty, np.eye(nx))
    Ct = (np.eye(nt) - np.eye(nt, k=-1)) / d.ht
    ref = np.kron(Ct, np.eye(nx * ny)) - np.kron(np.eye(nt), lap)
    np.testing.assert_allclose(D, ref, rtol=1e-13, atol=1e-10)
    # textbook eigenvalues of the 1-D second difference
    ev = np.sort(np.linalg.eigvalsh(-Tx))
    k = np.arange(1, nx + 1)
    np.testing.assert_allclose(ev, np.sort(4 * np.sin(k * np.pi / (2 * (nx + 1))) ** 2 / d.hx ** 2),
                               rtol=1e-12)


@pytest.mark.parametrize("var", [False, True])
def test_linewise_apply_matches_dense_assembly(var):
    w = tiny(var=var)
    d = op.disc_from(w)
    D = op.assemble_D(d)
    v = W.random_field(w.shape, 11)
    np.testing.assert_allclose(op.apply_D(d, v).ravel(), D @ v.ravel(), rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(op.apply_DT(d, v).ravel(), D.T @ v.ravel(), rtol=1e-12, atol=1e-9)
    Ds = op.assemble_D_sparse(d).toarray()
    np.testing.assert_allclose(Ds, D, rtol=1e-14, atol=1e-12)


def test_sampled_rows_match_apply():
    w = tiny(nx=9, ny=8, nt=3)
    d = op.disc_from(w)
    v = W.random_field(w.shape, 5)
    full = op.apply_D(d, v)
    pts = [(0, 0, 0), (2, 7, 8), (1, 3, 4), (2, 0, 8)]
    np.testing.assert_allclose(op.sampled_D(d, v, pts), [full[p] for p in pts], rtol=1e-12)


@pytest.mark.parametrize("var", [False, True])
def test_sampled_rows_match_assembled_matrix(var):
    """Rows of D and of D^T at single points (used for the full-size GPU
    checks) against the dense Kronecker assembly of eq. (4.9)."""
    w = tiny(nx=9, ny=8, nt=3, var=var)
    d = op.disc_from(w)
    v = W.random_field(w.shape, 6)
    D = op.assemble_D(d)
    pts = [(0, 0, 0), (2, 7, 8), (1, 3, 4), (2, 0, 8), (0, 7, 0), (1, 1, 7)]
    idx = [(t * w.ny + j) * w.nx + i for t, j, i in pts]
    np.testing.assert_allclose(op.sampled_D(d, v, pts), (D @ v.ravel())[idx], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(op.sampled_DT(d, v, pts), (D.T @ v.ravel())[idx], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("var", [False, True])
def test_m_matrix_and_positive_symmetric_part(var):
    w = tiny(var=var)
    d = op.disc_from(w)
    D = op.assemble_D(d)
    off = D - np.diag(np.diag(D))
    assert np.all(off <= 1e-12)  # Z-matrix
    Dinv = np.linalg.inv(D)
    assert np.all(Dinv >= -1e-12)  # inverse-nonnegative: an M-matrix
    assert np.min(np.linalg.eigvalsh(D + D.T)) > 0


def test_time_coupling_is_backward_difference():
    w = tiny(var=False)
    d = op.disc_from(w)
    v = np.zeros(w.shape)
    v[:] = np.arange(1, w.nt + 1)[:, None, None] ** 2  # spatially constant
    Ev = op.apply_E(d, v)
    np.testing.assert_allclose(Ev[:, 0, 0], np.diff(np.r_[0.0, np.arange(1, w.nt + 1) ** 2]) / d.ht)
    ETv = op.apply_ET(d, v)
    tv = np.arange(1, w.nt + 1) ** 2.0
    np.testing.assert_allclose(ETv[:, 0, 0], (tv - np.r_[tv[1:], 0.0]) / d.ht)


def test_psi_is_the_smallest_step_power():
    w = W.small()
    d = op.disc_from(w)
    assert op.psi_scale(d) == min(1 / 8, (1 / 17) ** 1.5, (1 / 17) ** 1.3)


@pytest.mark.parametrize("var", [False, True])
def test_time_stepping_solver_inverts_D(var):
    w = tiny(var=var)
    d = op.disc_from(w)
    D = op.assemble_D(d)
    S = op.DSolver(d)
    f = W.random_field((w.N, 3), 4)
    np.testing.assert_allclose(D @ S.solve(f), f, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(D.T @ S.solve(f, trans=True), f, rtol=1e-10, atol=1e-10)
