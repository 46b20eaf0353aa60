"""Pins for the diagonally scaled preconditioner Delta S~^{-1} Delta of
variable-coefficient problems (precond_kind = 2; the remark closing Sec. 4,
a diagonal times structured form; eq. (3.9) for S, eq. (3.10) for S~)."""
import numpy as np
import pytest

import workloads as W
from oracle import admm
from oracle import operator as op
from oracle import precond as pc


def var_case(nx=6, ny=5, nt=4, **kw):
    """Coefficients varying in x and y, trapezoidal objective weights (the
    last slice's M_y, M_p differ) and, by default, a Caputo time order (every
    time level couples to the later ones)."""
    w = W.small(nx=nx, ny=ny, nt=nt).replace(obj_weights=1, alpha_t=kw.pop("alpha_t", 0.6), **kw)
    rng = np.random.Generator(np.random.PCG64(11))
    w.dplus = 0.5 + rng.uniform(size=(ny, nx))
    w.dminus = 0.3 + rng.uniform(size=(ny, nx))
    return w


@pytest.mark.parametrize("alpha_t", [1.0, 0.6])
def test_diag_S_equals_dense_assembly(alpha_t):
    w = var_case(alpha_t=alpha_t)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    plane = w.nx * w.ny
    D = op.assemble_D(d)  # dense, a separate assembly from the sparse one diag_S uses
    S = np.diag(np.repeat(sc.My, plane)) + sc.psi ** 2 * D.T @ np.diag(1.0 / np.repeat(sc.Mp, plane)) @ D
    dS = pc.diag_S(w, d, sc.My, sc.Mp, sc.psi)
    np.testing.assert_allclose(dS.ravel(), np.diag(S), rtol=1e-13)


def test_diag_S_equals_probing_of_matrix_free_S():
    """e_i^T S e_i through the matrix-free operator (Toeplitz line products, no
    assembly) at sampled points, edges and corners included."""
    w = var_case(nx=9, ny=7, nt=5)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    dS = pc.diag_S(w, d, sc.My, sc.Mp, sc.psi)
    rng = np.random.Generator(np.random.PCG64(3))
    pts = [(0, 0, 0), (w.nt - 1, w.ny - 1, w.nx - 1), (2, 0, 8), (4, 6, 0)]
    pts += [tuple(int(rng.integers(n)) for n in (w.nt, w.ny, w.nx)) for _ in range(8)]
    for k, j, i in pts:
        e = np.zeros(w.shape)
        e[k, j, i] = 1.0
        assert abs(admm.apply_S(d, sc, e)[k, j, i] - dS[k, j, i]) <= 1e-13 * dS[k, j, i], (k, j, i)


def test_scaled_preconditioner_is_spd_and_unit_at_constant_diagonal():
    w = var_case(nx=6, ny=4, nt=3)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    tab = pc.precond_tables(w, d)
    delta = pc.scaling_factor(pc.diag_S(w, d, sc.My, sc.Mp, sc.psi))
    n = int(np.prod(w.shape))
    P = np.stack([pc.apply_precond_scaled(tab, delta, e.reshape(w.shape)).ravel() for e in np.eye(n)], axis=1)
    np.testing.assert_allclose(P, P.T, rtol=1e-12, atol=1e-14 * np.abs(P).max())
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0
    # a constant diagonal gives Delta = 1: the scaled form is S~ itself
    one = pc.scaling_factor(np.full(w.shape, 3.7))
    r = np.random.Generator(np.random.PCG64(5)).standard_normal(w.shape)
    np.testing.assert_allclose(pc.apply_precond_scaled(tab, one, r), pc.apply_precond(tab, r), rtol=1e-14)


def test_pcg_with_scaled_preconditioner_solves_S():
    """Same x-step solution as a dense solve of S x = b, with fewer PCG
    iterations than S~ at high coefficient contrast (d+ = 1 + 0.9 sin 2 pi x)."""
    w = W.headline(nx=24, ny=24, nt=8)
    w.dplus = W.coef_sine_x(24, 24, amp=0.9)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    tab = pc.precond_tables(w, d)
    delta = pc.scaling_factor(pc.diag_S(w, d, sc.My, sc.Mp, sc.psi))
    b = np.random.Generator(np.random.PCG64(9)).standard_normal(w.shape)
    A = lambda v: admm.apply_S(d, sc, v)
    x2, it2, _, ok2 = admm.pcg(A, lambda r: pc.apply_precond_scaled(tab, delta, r), b, np.zeros(w.shape), 1e-12, 500)
    x0, it0, _, ok0 = admm.pcg(A, lambda r: pc.apply_precond(tab, r), b, np.zeros(w.shape), 1e-12, 500)
    assert ok2 and ok0
    plane = w.nx * w.ny
    D = op.assemble_D(d)
    S = np.diag(np.repeat(sc.My, plane)) + sc.psi ** 2 * D.T @ np.diag(1.0 / np.repeat(sc.Mp, plane)) @ D
    x = np.linalg.solve(S, b.ravel()).reshape(w.shape)
    assert np.linalg.norm(x2 - x) <= 1e-10 * np.linalg.norm(x)
    assert it2 < it0, (it2, it0)


def test_admm_with_scaled_preconditioner_same_iterates():
    """The preconditioner changes only the Krylov path: ADMM iterates agree
    with S~'s to the Krylov tolerance."""
    w = W.small(nx=12, ny=10, nt=6).replace(krylov_tol=1e-12)
    w.dplus = W.coef_sine_x(12, 10, amp=0.9)
    a = admm.admm_solve(w, iters=6)
    b = admm.admm_solve(w.replace(precond_kind=2), iters=6)
    for k in ("y", "u", "p"):
        ref = getattr(a, k)
        assert np.linalg.norm(getattr(b, k) - ref) <= 1e-9 * max(np.linalg.norm(ref), 1e-300), k
    with pytest.raises(ValueError):
        admm.admm_solve(w.replace(precond_kind=2), iters=1, solver="minres")
