"""Pins for the saddle-point route of Sec. 3.3.1: preconditioned MINRES on the
merged x-step system (3.8) with the block-diagonal preconditioner K~ of
eq. (3.12)."""
import numpy as np
import pytest

import workloads as W
from oracle import admm, kkt, precond
from oracle import operator as op


def tiny(**kw):
    w = W.small(nx=5, ny=4, nt=3).replace(**kw)
    w.dplus = W.coef_sine_x(5, 4)
    return w


def rand_tuple(w, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return tuple(rng.standard_normal(w.shape) for _ in range(3))


def dense(fn, w):
    """Dense matrix of a map on (y, u, p) tuples."""
    N = w.N
    cols = []
    for k in range(3 * N):
        e = np.zeros(3 * N)
        e[k] = 1.0
        X = tuple(e[i * N:(i + 1) * N].reshape(w.shape) for i in range(3))
        cols.append(np.concatenate([f.ravel() for f in fn(X)]))
    return np.stack(cols, axis=1)


def flat(X):
    return np.concatenate([f.ravel() for f in X])


def setup(w):
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    tab = precond.precond_tables(w, d)
    K = lambda X: admm.apply_K(d, sc, w, X)
    M = lambda R: admm.apply_Kt_inv(tab, sc, R)
    return d, sc, tab, K, M


def test_K_is_the_merged_system_and_Kt_is_spd():
    w = tiny(ctrl_sign=-1.0, obj_weights=1, rho=1.3, delta=0.6)
    d, sc, tab, K, M = setup(w)
    Kd = dense(K, w)
    assert np.allclose(Kd, Kd.T, atol=1e-12)
    # the block solve of (3.8) is K's solve (its right-hand side, g = 0)
    zy, zu, p, wy, wu = (rand_tuple(w, 1) + rand_tuple(w, 2))[:5]
    y_ref, u_ref, p_ref = admm.xstep_block_solve(w, w.yhat, zy, zu, p, wy, wu)
    rho, delta = w.rho, w.delta
    J1 = admm.tcol(sc.wts)
    Ry = rho * (J1 * w.yhat - sc.e_y * wy + sc.e_y ** 2 * zy / delta) + (1 - rho) * admm.apply_BT(d, sc, p)
    Ru = rho * (-sc.e_u * wu + sc.e_u ** 2 * zu / delta) + (1 - rho) * sc.k_u * p
    sol = np.linalg.solve(Kd, flat((Ry, Ru, -(delta / rho) * p)))
    assert kkt.rel(sol, flat((y_ref, u_ref, p_ref))) < 1e-12
    Md = dense(M, w)
    Md = 0.5 * (Md + Md.T)
    assert np.linalg.eigvalsh(Md).min() > 0


@pytest.mark.parametrize("kind", [0, 1])
def test_minres_solves_the_merged_system(kind):
    w = tiny(ctrl_sign=-1.0, rho=0.9, delta=0.5, precond_kind=kind)
    d, sc, tab, K, M = setup(w)
    b = rand_tuple(w, 3)
    x, it, relres, conv = admm.minres(K, M, b, tuple(np.zeros(w.shape) for _ in range(3)), 1e-13, 500)
    assert conv and it < 3 * w.N
    ref = np.linalg.solve(dense(K, w), flat(b))
    assert kkt.rel(flat(x), ref) < 1e-10


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_minres_iterate_minimises_the_residual_over_the_krylov_space(k):
    """After k steps from x0 the iterate minimises |b - K x| in the K~^{-1}
    norm over x0 + span{t, (K~^{-1} K) t, ...}, t = K~^{-1}(b - K x0): brute
    force by least squares on an orthonormalised Krylov basis."""
    w = tiny(ctrl_sign=-1.0, obj_weights=1)
    d, sc, tab, K, M = setup(w)
    Kd, Minv = dense(K, w), dense(M, w)
    Minv = 0.5 * (Minv + Minv.T)
    b = rand_tuple(w, 4)
    x0 = rand_tuple(w, 5)
    xk, it, _, _ = admm.minres(K, M, b, x0, 0.0, k)
    assert it == k
    r0 = flat(b) - Kd @ flat(x0)
    T = [Minv @ r0]
    for _ in range(k - 1):
        T.append(Minv @ (Kd @ T[-1]))
    Q, _ = np.linalg.qr(np.stack(T, axis=1))
    L = np.linalg.cholesky(Minv)  # |r|_{M^-1}^2 = |L^T r|^2
    c, *_ = np.linalg.lstsq(L.T @ Kd @ Q, L.T @ r0, rcond=None)
    ref = flat(x0) + Q @ c
    assert np.max(np.abs(flat(xk) - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_exact_schur_block_gives_the_saddle_point_intervals():
    """With circulant constraints (C_3 itself), scalar blocks and the exact
    Schur complement in the third block, the eigenvalues of K~^{-1} K lie in
    [-1, (1 - sqrt 5)/2] and [1, (1 + sqrt 5)/2]: the intervals of a
    block-diagonal preconditioner with the exact Schur complement for a
    saddle-point matrix whose (2,2) block is negative semi-definite."""
    w = W.small(nx=6, ny=5, nt=4).replace(prox=1, rho=0.9, delta=0.7)
    d, sc, tab, _, M = setup(w)
    Cx, Cy, Ct = (precond.circulant(tab["col_x"]), precond.circulant(tab["col_y"]), precond.circulant(tab["col_t"]))
    nx, ny, nt, N = w.nx, w.ny, w.nt, w.N
    C3 = tab["psi"] * (np.kron(Ct, np.eye(nx * ny)) - np.kron(np.eye(nt), np.kron(Cy, np.eye(nx)))
                       - np.kron(np.eye(nt * ny), Cx))
    I = np.eye(N)
    assert np.allclose(sc.My, tab["a"]) and np.allclose(sc.Mp, tab["mbar_p"])
    Kc = np.block([[sc.My[0] * I, np.zeros((N, N)), C3.T], [np.zeros((N, N)), sc.Mu[0] * I, sc.k_u * I],
                   [C3, sc.k_u * I, -(w.delta / w.rho) * I]])
    Md = dense(M, w)
    ev = np.linalg.eigvals(Md @ Kc).real
    lo, hi = (1 - np.sqrt(5)) / 2, (1 + np.sqrt(5)) / 2
    neg, pos = ev[ev < 0], ev[ev > 0]
    assert len(neg) == N and len(pos) == 2 * N
    assert neg.min() >= -1 - 1e-10 and neg.max() <= lo + 1e-10
    assert pos.min() >= 1 - 1e-10 and pos.max() <= hi + 1e-10


def test_admm_with_minres_matches_admm_with_pcg():
    """Both x-step solvers reach the same fixed point: with tight Krylov
    tolerances their ADMM iterates agree."""
    w = W.small_mixed(nx=8, ny=6, nt=4, obj_weights=1, krylov_tol=1e-13)
    a = admm.admm_solve(w, iters=30)
    b = admm.admm_solve(w, iters=30, solver="minres")
    for k in ("y", "u", "zy", "zu", "p", "wy", "wu"):
        assert kkt.rel(getattr(b, k), getattr(a, k)) < 1e-9, k
    r = admm.admm_solve(w.replace(krylov_tol=1e-10, admm_tol=1e-8), solver="minres")
    assert r.converged and kkt.polish(w, r.zy, r.zu)["ok"]
