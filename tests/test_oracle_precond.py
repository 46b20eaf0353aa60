"""Pins for the T. Chan circulants and the preconditioner S~ (Sec. 5, eq. (5.2); eq. (3.10))."""
import numpy as np
import pytest

import workloads as W
from oracle import operator as op
from oracle import precond as pc


def random_toeplitz(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    t = rng.standard_normal(2 * n - 1)  # t_{-(n-1)} .. t_{n-1}
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return t[(i - j) + n - 1]


@pytest.mark.parametrize("n", [5, 16, 33])
def test_tchan_is_frobenius_optimal(n):
    T = random_toeplitz(n, n)
    c = pc.tchan_column(T)
    # brute force: least-squares fit of sum_i c_i P_i to T over all circulants
    basis = np.stack([pc.circulant(np.eye(n)[i]).ravel() for i in range(n)], axis=1)
    c_ls, *_ = np.linalg.lstsq(basis, T.ravel(), rcond=None)
    np.testing.assert_allclose(c, c_ls, rtol=1e-12, atol=1e-13)
    # equivalently the mean of each wrapped diagonal
    wrapped = np.array([np.mean([T[(i + j) % n, j] for j in range(n)]) for i in range(n)])
    np.testing.assert_allclose(c, wrapped, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("n", [4, 12, 31])
def test_circulant_eigenvalues_are_dft_of_first_column(n):
    rng = np.random.Generator(np.random.PCG64(n))
    c = rng.standard_normal(n)
    lam = pc.dft_eigenvalues(c)
    np.testing.assert_allclose(lam, np.fft.fft(c), rtol=1e-11, atol=1e-12)
    C = pc.circulant(c)
    m = np.arange(n)
    for k in range(n):
        v = np.exp(2j * np.pi * k * m / n)
        np.testing.assert_allclose(C @ v, lam[k] * v, atol=1e-11)


@pytest.mark.parametrize("a", [1.1, 1.5, 1.9])
@pytest.mark.parametrize("n", [32, 64])
def test_riesz_tchan_spectrum(a, n):
    h = 1.0 / (n + 1)
    L = pc.mean_line_operator(a, h, n, 1.0, 1.0)
    lam = pc.dft_eigenvalues(pc.tchan_column(L))
    assert np.max(np.abs(lam.imag)) < 1e-9 * np.max(np.abs(lam))
    ev = np.linalg.eigvalsh(L)
    assert np.all(lam.real < 0)
    assert np.all(lam.real >= ev.min() - 1e-9 * abs(ev.min()))
    assert np.all(lam.real <= ev.max() + 1e-9 * abs(ev.min()))


def test_time_tchan_column_and_spectrum():
    nt, ht = 8, 1 / 8
    c = pc.tchan_column(op.time_matrix(nt, ht))
    np.testing.assert_allclose(c, np.r_[1.0, -(nt - 1) / nt, np.zeros(nt - 2)] / ht, rtol=1e-15)
    lam = pc.dft_eigenvalues(c)
    assert abs(np.min(np.abs(lam)) - 1.0 / (nt * ht)) < 1e-12


def _tiny(var):
    w = W.small(nx=6, ny=5, nt=4).replace(alpha=1.4, beta=1.6, rho=1.3, delta=0.7, gamma=1e-3)
    if var:
        w.dplus = W.coef_sine_x(6, 5)
    return w


@pytest.mark.parametrize("var", [False, True])
def test_precond_matches_dense_schur_approximation(var):
    w = _tiny(var)
    d = op.disc_from(w)
    tab = pc.precond_tables(w, d)
    # assemble C_3(B) of eq. (5.2) from the 1-D T. Chan circulants (Kronecker)
    Cx, Cy, Ct = (pc.circulant(tab["col_x"]), pc.circulant(tab["col_y"]), pc.circulant(tab["col_t"]))
    nx, ny, nt = w.nx, w.ny, w.nt
    C3 = tab["psi"] * (np.kron(Ct, np.eye(nx * ny)) - np.kron(np.eye(nt), np.kron(Cy, np.eye(nx)))
                       - np.kron(np.eye(nt * ny), Cx))
    S_t = tab["a"] * np.eye(w.N) + C3.T @ C3 / tab["mbar_p"]
    r = W.random_field(w.shape, 4)
    z = pc.apply_precond(tab, r)
    np.testing.assert_allclose(S_t @ z.ravel(), r.ravel(), rtol=1e-11, atol=1e-11)
    # separable eigenvalues (eq. (5.2)) against the assembled C_3 on Fourier vectors
    s = pc.precond_symbol(tab)
    assert np.all(s > 0)
    t, j, i = np.meshgrid(np.arange(nt), np.arange(ny), np.arange(nx), indexing="ij")
    for (kt, ky, kx) in [(0, 0, 0), (1, 2, 3), (3, 4, 5)]:
        v = np.exp(2j * np.pi * (kt * t / nt + ky * j / ny + kx * i / nx)).ravel()
        lam = tab["psi"] * (tab["lam_t"][kt] - tab["lam_y"][ky] - tab["lam_x"][kx])
        np.testing.assert_allclose(C3 @ v, lam * v, atol=1e-9 * abs(lam))


def test_coefficient_mean_of_sine_field_is_one():
    d = W.coef_sine_x(256, 256)
    assert abs(np.mean(d) - 1.0) < 1e-14


def _c3(tab, w):
    Cx, Cy, Ct = (pc.circulant(tab["col_x"]), pc.circulant(tab["col_y"]), pc.circulant(tab["col_t"]))
    nx, ny, nt = w.nx, w.ny, w.nt
    return tab["psi"] * (np.kron(Ct, np.eye(nx * ny)) - np.kron(np.eye(nt), np.kron(Cy, np.eye(nx)))
                         - np.kron(np.eye(nt * ny), Cx))


@pytest.mark.parametrize("var", [False, True])
@pytest.mark.parametrize("prox", [0, 1])
def test_matching_precond_matches_dense_eq_3_11(var, prox):
    """precond_kind = 1 solves with S^ = D^ M2~^{-1} D^*, D^ = C_3^* + (M1~ M2~)^{1/2},
    assembled densely from the 1-D T. Chan circulants."""
    w = _tiny(var).replace(precond_kind=1, prox=prox, rho=0.9 if prox else 1.3)
    tab = pc.precond_tables(w, op.disc_from(w))
    assert tab["kind"] == 1
    C3 = _c3(tab, w)
    c = np.sqrt(tab["a"] * tab["mbar_p"])
    Dh = C3.T + c * np.eye(w.N)
    S_h = Dh @ Dh.T / tab["mbar_p"]
    r = W.random_field(w.shape, 5)
    z = pc.apply_precond(tab, r)
    np.testing.assert_allclose(S_h @ z.ravel(), r.ravel(), rtol=1e-11, atol=1e-11)


def test_matching_theorem_interval_for_circulant_constraints():
    """Thm 3.5 (second part): with scalar (1,1)/(2,2) blocks and a constraint
    matrix whose symmetric part is positive semi-definite, S^{-1} S has its
    eigenvalues in [1/2, 1].  Taking the constraint matrix to be C_3 itself,
    S is exactly S~ = a I + C_3^T C_3 / mbar_p."""
    w = _tiny(False)
    tab = pc.precond_tables(w, op.disc_from(w))
    C3 = _c3(tab, w)
    assert np.linalg.eigvalsh(C3 + C3.T).min() >= -1e-12  # D + D^* positive semi-definite
    S = tab["a"] * np.eye(w.N) + C3.T @ C3 / tab["mbar_p"]
    c = np.sqrt(tab["a"] * tab["mbar_p"])
    Dh = C3.T + c * np.eye(w.N)
    S_h = Dh @ Dh.T / tab["mbar_p"]
    ev = np.linalg.eigvals(np.linalg.solve(S_h, S)).real
    assert ev.min() >= 0.5 - 1e-12 and ev.max() <= 1.0 + 1e-12
    # and the interval is not trivially [1, 1]: S^ differs from S~
    assert ev.min() < 0.99


@pytest.mark.parametrize("nx", [6, 7])
@pytest.mark.parametrize("kind", [0, 1])
def test_rz_from_the_half_spectrum(nx, kind):
    """(r, S~^{-1} r) equals sum |R_k|^2 / (s_k N) over the half spectrum
    kx = 0..nx/2, with columns other than 0 and nx/2 counted twice: the
    symbol is even (s_{-k} = s_k) also when the mean coefficients differ
    (non-symmetric circulants).  This is how the GPU forms (r, z) in PCG."""
    ny, nt = 5, 4
    w = W.small(nx=nx, ny=ny, nt=nt).replace(alpha=1.4, beta=1.6, rho=1.3, delta=0.7, gamma=1e-3,
                                             precond_kind=kind)
    w.dplus = np.full((ny, nx), 2.0)  # mean d+ = 2, d- = 1: L_x, L_y not symmetric
    tab = pc.precond_tables(w, op.disc_from(w))
    s = pc.precond_symbol(tab)
    neg = s[(-np.arange(nt)) % nt][:, (-np.arange(ny)) % ny][:, :, (-np.arange(nx)) % nx]
    np.testing.assert_allclose(neg, s, rtol=1e-13)
    assert not np.allclose(tab["lam_x"].imag, 0.0)  # the circulant really is non-symmetric
    r = W.random_field(w.shape, 11)
    direct = float(np.sum(r * pc.apply_precond(tab, r)))
    R = np.fft.fftn(r)
    H = nx // 2 + 1
    wt = np.full(H, 2.0)
    wt[0] = 1.0
    if nx % 2 == 0:
        wt[-1] = 1.0
    half = float(np.sum(wt * np.abs(R[:, :, :H]) ** 2 / s[:, :, :H])) / r.size
    assert abs(half - direct) <= 1e-13 * abs(direct)
    # a weight of 2 on the Nyquist column (or 1 on the others) is visibly wrong
    bad = wt.copy()
    bad[-1] = 3.0 - bad[-1]
    wrong = float(np.sum(bad * np.abs(R[:, :, :H]) ** 2 / s[:, :, :H])) / r.size
    assert abs(wrong - direct) > 1e-6 * abs(direct)
