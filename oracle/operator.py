"""The discretised fractional-diffusion constraint matrix D -- oracle, test infrastructure.

Sec. 4: D = C_t (x) I - I (x) (L_x (+) L_y), eq. (4.9), with
  * time: the non-shifted Grünwald (Caputo) matrix of eq. (4.5) of order
    alpha_t in (0, 1]: lower-triangular Toeplitz with first column
    g_k(alpha_t) / h_t^alpha_t; at alpha_t = 1 the weights are (1, -1, 0, ...)
    and C_t = (I - Z) / h_t is implicit Euler (Z the sub-diagonal shift);
    y(t=0) = 0;
  * space: the shifted (p = 1) Grünwald matrix of eq. (4.6),
    G[i, j] = g_{i-j+1} for i-j+1 >= 0, and the two-sided operator
    L_a = (c_a / h^a) (diag(d+) G + diag(d-) G^T), c_a the Riesz factor of
    eq. (4.7).  With d+ = d- = 1 this is exactly the paper's Riesz matrix;
    the row scaling by a coefficient field is the variable-coefficient
    reading (coefficient outside the derivative).
Fields are arrays of shape (nt, ny, nx) (x fastest).  Products along x use
G on the last axis, products along y on the middle axis: dense matrix
products, no FFT.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .grunwald import riesz_factor, weights


@dataclasses.dataclass
class Disc:
    nx: int
    ny: int
    nt: int
    hx: float
    hy: float
    ht: float
    alpha: float
    beta: float
    dplus: np.ndarray  # (ny, nx)
    dminus: np.ndarray  # (ny, nx)
    alpha_t: float = 1.0  # order of the time derivative


def disc_from(w) -> Disc:
    """Mesh sizes h_x = 1/(nx+1), h_y = 1/(ny+1), h_t = T/nt (Sec. 6.1 grid)."""
    ones = np.ones((w.ny, w.nx))
    dp = ones if w.dplus is None else np.asarray(w.dplus, dtype=np.float64)
    dm = ones if w.dminus is None else np.asarray(w.dminus, dtype=np.float64)
    return Disc(nx=w.nx, ny=w.ny, nt=w.nt, hx=1.0 / (w.nx + 1), hy=1.0 / (w.ny + 1),
                ht=w.T / w.nt, alpha=w.alpha, beta=w.beta, dplus=dp, dminus=dm,
                alpha_t=getattr(w, "alpha_t", 1.0))


def shifted_grunwald(a: float, n: int, g: np.ndarray | None = None) -> np.ndarray:
    """n x n left shifted Grünwald matrix of eq. (4.6) without the 1/h^a factor:
    entry (i, j) is g_{i-j+1} when i-j+1 >= 0, else 0.  `g` overrides the
    weights (used with derivative weights)."""
    if g is None:
        g = weights(a, n)
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    k = i - j + 1
    return np.where(k >= 0, g[np.clip(k, 0, n)], 0.0)


def time_matrix(nt: int, ht: float, alpha_t: float = 1.0) -> np.ndarray:
    """The Caputo matrix of eq. (4.5): entry (k, m) is g_{k-m}(alpha_t) / h_t^alpha_t
    for k >= m.  Order 1 is implicit Euler, (I - Z) / h_t."""
    if alpha_t == 1.0:
        return (np.eye(nt) - np.eye(nt, k=-1)) / ht
    g = weights(alpha_t, nt - 1)
    k = np.arange(nt)[:, None] - np.arange(nt)[None, :]
    return np.where(k >= 0, g[np.clip(k, 0, nt - 1)], 0.0) / ht ** alpha_t


# --- line-wise applies -------------------------------------------------------
def apply_E(d: Disc, v):
    """C_t along every t-line: implicit Euler as a difference, a fractional
    order as the dense lower-triangular product."""
    if d.alpha_t == 1.0:
        out = v.copy()
        out[1:] -= v[:-1]
        return out / d.ht
    return np.tensordot(time_matrix(d.nt, d.ht, d.alpha_t), v, axes=([1], [0]))


def apply_ET(d: Disc, v):
    if d.alpha_t == 1.0:
        out = v.copy()
        out[:-1] -= v[1:]
        return out / d.ht
    return np.tensordot(time_matrix(d.nt, d.ht, d.alpha_t).T, v, axes=([1], [0]))


def apply_Lx(d: Disc, v, transpose=False):
    """L_x along every x-line (t, j): row scaling by d+/d- of that line."""
    G = shifted_grunwald(d.alpha, d.nx)
    s = riesz_factor(d.alpha) / d.hx ** d.alpha
    if not transpose:
        # (G v)_i = sum_k G[i,k] v_k ; (G^T v)_i = sum_k G[k,i] v_k
        return s * (d.dplus * (v @ G.T) + d.dminus * (v @ G))
    return s * ((d.dplus * v) @ G + (d.dminus * v) @ G.T)


def apply_Ly(d: Disc, v, transpose=False):
    """L_y along every y-line (t, i)."""
    G = shifted_grunwald(d.beta, d.ny)
    s = riesz_factor(d.beta) / d.hy ** d.beta
    if not transpose:
        return s * (d.dplus * np.matmul(G, v) + d.dminus * np.matmul(G.T, v))
    return s * (np.matmul(G.T, d.dplus * v) + np.matmul(G, d.dminus * v))


def apply_D(d: Disc, v):
    """D v = C_t v - L_x v - L_y v (eq. (4.9))."""
    return apply_E(d, v) - apply_Lx(d, v) - apply_Ly(d, v)


def apply_DT(d: Disc, v):
    """D^T v."""
    return apply_ET(d, v) - apply_Lx(d, v, True) - apply_Ly(d, v, True)


# --- dense assembly (small grids) -------------------------------------------
def line_matrix(a, h, n, dp_line, dm_line, g=None):
    G = shifted_grunwald(a, n, g)
    return riesz_factor(a) / h ** a * (np.diag(dp_line) @ G + np.diag(dm_line) @ G.T)


def assemble_D(d: Disc) -> np.ndarray:
    """Dense D by Kronecker assembly of eq. (4.9); index (t*ny + j)*nx + i."""
    nx, ny, nt = d.nx, d.ny, d.nt
    M = nx * ny
    Lx = np.zeros((M, M))
    Ly = np.zeros((M, M))
    for j in range(ny):
        Lj = line_matrix(d.alpha, d.hx, nx, d.dplus[j, :], d.dminus[j, :])
        Lx[j * nx:(j + 1) * nx, j * nx:(j + 1) * nx] = Lj
    for i in range(nx):
        Li = line_matrix(d.beta, d.hy, ny, d.dplus[:, i], d.dminus[:, i])
        idx = np.arange(ny) * nx + i
        Ly[np.ix_(idx, idx)] = Li
    return np.kron(time_matrix(nt, d.ht, d.alpha_t), np.eye(M)) - np.kron(np.eye(nt), Lx + Ly)


def assemble_D_sparse(d: Disc):
    """The same matrix as scipy.sparse CSR (used for the active-set polish)."""
    import scipy.sparse as sp

    nx, ny, nt = d.nx, d.ny, d.nt
    M = nx * ny
    blocks_x = [sp.csr_matrix(line_matrix(d.alpha, d.hx, nx, d.dplus[j, :], d.dminus[j, :]))
                for j in range(ny)]
    Lx = sp.block_diag(blocks_x, format="csr")
    rows, cols, vals = [], [], []
    for i in range(nx):
        Li = line_matrix(d.beta, d.hy, ny, d.dplus[:, i], d.dminus[:, i])
        jj, kk = np.nonzero(Li)
        rows.append(jj * nx + i)
        cols.append(kk * nx + i)
        vals.append(Li[jj, kk])
    Ly = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(M, M))
    Ct = sp.csr_matrix(time_matrix(nt, d.ht, d.alpha_t))
    return (sp.kron(Ct, sp.identity(M)) - sp.kron(sp.identity(nt), Lx + Ly)).tocsr()


class DSolver:
    """Direct solves with D and D^T by time stepping: D is block lower
    triangular with blocks c_{k-m} I below the diagonal (c the first column of
    the time matrix; block lower bidiagonal for implicit Euler) and diagonal
    blocks A = c_0 I - (L_x (+) L_y).  One dense LU of the 2-D block A; step k
    moves the history sum to the right-hand side.  Right-hand sides are (N,)
    or (N, m) arrays in the (t*ny + j)*nx + i ordering."""

    def __init__(self, d: Disc):
        import scipy.linalg as sla

        self.d = d
        M = d.nx * d.ny
        Lx = np.zeros((M, M))
        Ly = np.zeros((M, M))
        for j in range(d.ny):
            Lx[j * d.nx:(j + 1) * d.nx, j * d.nx:(j + 1) * d.nx] = line_matrix(
                d.alpha, d.hx, d.nx, d.dplus[j, :], d.dminus[j, :])
        for i in range(d.nx):
            idx = np.arange(d.ny) * d.nx + i
            Ly[np.ix_(idx, idx)] = line_matrix(d.beta, d.hy, d.ny, d.dplus[:, i], d.dminus[:, i])
        self.c = time_matrix(d.nt, d.ht, d.alpha_t)[:, 0].copy()
        A = self.c[0] * np.eye(M) - Lx - Ly
        self.lu = sla.lu_factor(A)
        self.M = M

    def solve(self, f, trans=False):
        import scipy.linalg as sla

        d, M = self.d, self.M
        f = np.asarray(f, dtype=np.float64)
        shp = f.shape
        F = f.reshape(d.nt, M, -1)
        X = np.empty_like(F)
        c = self.c
        if not trans:
            for k in range(d.nt):
                rhs = F[k] - sum(c[k - m] * X[m] for m in range(k) if c[k - m] != 0.0)
                X[k] = sla.lu_solve(self.lu, rhs)
        else:
            for k in range(d.nt - 1, -1, -1):
                rhs = F[k] - sum(c[m - k] * X[m] for m in range(k + 1, d.nt) if c[m - k] != 0.0)
                X[k] = sla.lu_solve(self.lu, rhs, trans=1)
        return X.reshape(shp)


def psi_scale(d: Disc) -> float:
    """psi = min{h_t^alpha_t, h_x^alpha, h_y^beta} (Sec. 5)."""
    return min(d.ht ** d.alpha_t, d.hx ** d.alpha, d.hy ** d.beta)


def sampled_D(d: Disc, v, points):
    """(D v) at the listed (t, j, i) points only, from the point's own row of D:
    its x-line, its y-line and its time history.  Cost O(nx + ny + nt) per point."""
    ga = weights(d.alpha, d.nx)
    gb = weights(d.beta, d.ny)
    sx = riesz_factor(d.alpha) / d.hx ** d.alpha
    sy = riesz_factor(d.beta) / d.hy ** d.beta
    ct = time_matrix(d.nt, d.ht, d.alpha_t)[:, 0]
    out = np.empty(len(points))
    for n, (t, j, i) in enumerate(points):
        # row i of G: entries g_{i-k+1} for k <= i+1 ; row i of G^T: g_{k-i+1} for k >= i-1
        k = np.arange(d.nx)
        rowG = np.where(i - k + 1 >= 0, ga[np.clip(i - k + 1, 0, d.nx)], 0.0)
        rowGT = np.where(k - i + 1 >= 0, ga[np.clip(k - i + 1, 0, d.nx)], 0.0)
        lx = sx * (d.dplus[j, i] * rowG @ v[t, j, :] + d.dminus[j, i] * rowGT @ v[t, j, :])
        k = np.arange(d.ny)
        rowG = np.where(j - k + 1 >= 0, gb[np.clip(j - k + 1, 0, d.ny)], 0.0)
        rowGT = np.where(k - j + 1 >= 0, gb[np.clip(k - j + 1, 0, d.ny)], 0.0)
        ly = sy * (d.dplus[j, i] * rowG @ v[t, :, i] + d.dminus[j, i] * rowGT @ v[t, :, i])
        out[n] = float(np.dot(ct[:t + 1], v[t::-1, j, i])) - lx - ly
    return out


def sampled_DT(d: Disc, v, points):
    """(D^T v) at the listed (t, j, i) points only, from row (t, j, i) of D^T
    (column of D): its x-line, its y-line and its later times.
    (L^T v)_i = c h^-a sum_k (G[k, i] d+_k + G[i, k] d-_k) v_k."""
    ga = weights(d.alpha, d.nx)
    gb = weights(d.beta, d.ny)
    sx = riesz_factor(d.alpha) / d.hx ** d.alpha
    sy = riesz_factor(d.beta) / d.hy ** d.beta
    ct = time_matrix(d.nt, d.ht, d.alpha_t)[:, 0]
    out = np.empty(len(points))
    for n, (t, j, i) in enumerate(points):
        k = np.arange(d.nx)
        colG = np.where(k - i + 1 >= 0, ga[np.clip(k - i + 1, 0, d.nx)], 0.0)  # G[k, i]
        rowG = np.where(i - k + 1 >= 0, ga[np.clip(i - k + 1, 0, d.nx)], 0.0)  # G[i, k]
        lx = sx * np.sum((colG * d.dplus[j, :] + rowG * d.dminus[j, :]) * v[t, j, :])
        k = np.arange(d.ny)
        colG = np.where(k - j + 1 >= 0, gb[np.clip(k - j + 1, 0, d.ny)], 0.0)
        rowG = np.where(j - k + 1 >= 0, gb[np.clip(j - k + 1, 0, d.ny)], 0.0)
        ly = sy * np.sum((colG * d.dplus[:, i] + rowG * d.dminus[:, i]) * v[t, :, i])
        out[n] = float(np.dot(ct[:d.nt - t], v[t:, j, i])) - lx - ly
    return out
