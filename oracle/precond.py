"""T. Chan circulants and the Schur-complement preconditioner -- oracle, test infrastructure.

Sec. 5: the T. Chan (Frobenius-optimal) circulant of a Toeplitz matrix T_n has
first column c_i = ((n-i) t_i + i t_{i-n}) / n (closed form under eq. (5.1)),
and its eigenvalues are the DFT of c (Thm 2.2).  The 3-level circulant
C_3(B) of eq. (5.2) has the separable eigenvalues
    Lambda = psi (lambda_t[k] - lambda_y[j] - lambda_x[i]).
Sec. 3.2, eq. (3.10): with circulant blocks and J_1 approximated by the
scalar jbar = 1 (the paper notes J is nearly a scaled identity, Sec. 4),
    S~ = rho (jbar + e_y^2/delta) I + C_3(B)^* C_3(B) / mbar_p,
    mbar_p = k_u^2 / (rho (gamma jbar + e_u^2/delta)) + delta/rho,
so S~ has eigenvalues s = a + |Lambda|^2 / mbar_p in the DFT basis.
Sec. 3.2.2, eq. (3.11): the matching approximation with the same blocks,
    S^ = D^ M2~^{-1} D^*,  D^ = C_3(B)^* + (M1~ M2~)^{1/2},  M1~ = a, M2~ = mbar_p,
is a circulant too, with eigenvalues |Lambda + sqrt(a mbar_p)|^2 / mbar_p
(precond_kind = 1).
Variable coefficients (the remark closing Sec. 4: circulants lose effect when
the coefficients vary, and a diagonal-times-structured form is the remedy the
paper points to) -- precond_kind = 2, read here as the symmetric diagonal
scaling of S~,
    P^{-1} = Delta S~^{-1} Delta,  Delta = (s0 / diag(S))^{1/2},
with diag(S) the exact diagonal of S = M_y + B^T M_p^{-1} B (eq. (3.9)) and s0
its mean over the grid (any constant gives the same PCG iterates).  Delta
carries the coefficient field's local size into the preconditioner; the
circulant keeps the mean-coefficient spectrum.

DFT convention: lambda_k = sum_m c_m exp(-2 pi i k m / n), computed here by the
explicit O(n^2) sum; the circulant acts as C x = F^{-1} diag(lambda) F x with
F[k, m] = exp(-2 pi i k m / n) and F^{-1} = conj(F) / n.  Variable
coefficients enter the preconditioner through their arithmetic means over
the interior nodes.
"""
from __future__ import annotations

import numpy as np

from .grunwald import riesz_factor
from .operator import Disc, psi_scale, shifted_grunwald, time_matrix


def tchan_column(T: np.ndarray) -> np.ndarray:
    """First column of the T. Chan circulant of the Toeplitz matrix T
    (t_k = T[k, 0] for k >= 0, t_{-k} = T[0, k])."""
    n = T.shape[0]
    c = np.empty(n, dtype=T.dtype)
    for i in range(n):
        t_i = T[i, 0]
        t_i_minus_n = T[0, n - i] if i > 0 else 0.0
        c[i] = ((n - i) * t_i + i * t_i_minus_n) / n
    return c


def dft_matrix(n: int) -> np.ndarray:
    """F[k, m] = exp(-2 pi i k m / n), with k*m reduced mod n first (exact)."""
    k = np.arange(n)
    return np.exp(-2j * np.pi * (np.outer(k, k) % n) / n)


def dft_eigenvalues(c: np.ndarray) -> np.ndarray:
    """lambda_k = sum_m c_m exp(-2 pi i k m / n), explicit sum."""
    return dft_matrix(len(c)) @ c


def circulant(c: np.ndarray) -> np.ndarray:
    """Dense circulant with first column c: C[i, j] = c[(i - j) mod n]."""
    n = len(c)
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return c[(i - j) % n]


def mean_line_operator(a, h, n, dbar_plus, dbar_minus):
    """Constant-coefficient (mean-coefficient) spatial Toeplitz matrix."""
    G = shifted_grunwald(a, n)
    return riesz_factor(a) / h ** a * (dbar_plus * G + dbar_minus * G.T)


def precond_tables(w, d: Disc):
    """Eigenvalue tables and scalars of S~ (Sec. 5, eq. (5.2); eq. (3.10))."""
    dbp = float(np.mean(d.dplus))
    dbm = float(np.mean(d.dminus))
    Lx = mean_line_operator(d.alpha, d.hx, d.nx, dbp, dbm)
    Ly = mean_line_operator(d.beta, d.hy, d.ny, dbp, dbm)
    Ct = time_matrix(d.nt, d.ht, d.alpha_t)
    col_x, col_y, col_t = tchan_column(Lx), tchan_column(Ly), tchan_column(Ct)
    lam_x = dft_eigenvalues(col_x)
    lam_y = dft_eigenvalues(col_y)
    lam_t = dft_eigenvalues(col_t)
    psi = psi_scale(d) if w.psi_scaling else 1.0
    e_y = 1.0
    e_u = psi if w.psi_scaling == 1 else 1.0
    k_u = psi * w.ctrl_sign
    jbar = 1.0
    cy, cu = jbar, w.gamma * jbar
    if getattr(w, "prox", 0):
        # Algorithm 2: the (1,1), (2,2) blocks are c_y I and c_u I exactly
        cy = w.prox_cy if w.prox_cy > 0 else jbar
        cu = w.prox_cu if w.prox_cu > 0 else w.gamma * jbar
    a = w.rho * (cy + e_y ** 2 / w.delta)
    mbar_p = k_u ** 2 / (w.rho * (cu + e_u ** 2 / w.delta)) + w.delta / w.rho
    return dict(lam_x=lam_x, lam_y=lam_y, lam_t=lam_t, col_x=col_x, col_y=col_y, col_t=col_t,
                psi=psi, a=a, mbar_p=mbar_p, kind=int(getattr(w, "precond_kind", 0)))


def precond_symbol(tab) -> np.ndarray:
    """s[k, j, i] = a + |Lam|^2 / mbar_p (S~, eq. (3.10)) or
    |Lam + sqrt(a mbar_p)|^2 / mbar_p (S^, eq. (3.11)), with
    Lam = psi (lam_t[k] - lam_y[j] - lam_x[i])."""
    lam = tab["psi"] * (tab["lam_t"][:, None, None] - tab["lam_y"][None, :, None]
                        - tab["lam_x"][None, None, :])
    if tab.get("kind", 0) == 1:
        return np.abs(lam + np.sqrt(tab["a"] * tab["mbar_p"])) ** 2 / tab["mbar_p"]
    return tab["a"] + np.abs(lam) ** 2 / tab["mbar_p"]


def apply_precond(tab, r: np.ndarray) -> np.ndarray:
    """z = S~^{-1} r with dense DFT matrices along each axis (no FFT)."""
    nt, ny, nx = r.shape
    Fx, Fy, Ft = dft_matrix(nx), dft_matrix(ny), dft_matrix(nt)
    R = r.astype(np.complex128) @ Fx.T  # along x
    R = np.matmul(Fy, R)  # along y
    R = np.tensordot(Ft, R, axes=([1], [0]))  # along t
    R = R / precond_symbol(tab)
    Z = np.tensordot(np.conj(Ft), R, axes=([1], [0])) / nt
    Z = np.matmul(np.conj(Fy), Z) / ny
    Z = Z @ np.conj(Fx).T / nx
    return Z.real.copy()


def diag_S(w, d: Disc, My, Mp, psi) -> np.ndarray:
    """Diagonal of S = M_y + B^T M_p^{-1} B with B = psi D (eq. (3.9), scaled
    form), as a field (nt, ny, nx): S_ii = M_y(t_i) + psi^2 sum_r D[r, i]^2 /
    M_p(t_r), the sum over the entries of column i of the assembled D
    (eq. (4.9)).  My, Mp: per time slice."""
    from .operator import assemble_D_sparse

    plane = d.nx * d.ny
    D = assemble_D_sparse(d)
    col = (D.multiply(D)).T @ np.repeat(1.0 / np.asarray(Mp, dtype=np.float64), plane)
    return (np.repeat(np.asarray(My, dtype=np.float64), plane) + psi ** 2 * col).reshape(d.nt, d.ny, d.nx)


def scaling_factor(dS: np.ndarray) -> np.ndarray:
    """Delta = (s0 / diag S)^{1/2}, s0 the mean of diag S (precond_kind = 2)."""
    return np.sqrt(float(np.mean(dS)) / dS)


def apply_precond_scaled(tab, delta: np.ndarray, r: np.ndarray) -> np.ndarray:
    """z = Delta S~^{-1} Delta r (precond_kind = 2)."""
    return delta * apply_precond(tab, delta * r)
