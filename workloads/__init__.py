"""Seeded synthetic inputs for the FDE-constrained optimal-control workloads.

This module is shared by the CPU oracle and the GPU path.  It holds problem
*descriptions* (grid sizes, fractional orders, bounds, regularisation) and the
seeded generators of the data fields (desired state, diffusion coefficients,
right-hand side).  It contains none of the method's arithmetic: no Grünwald
weights, no operators, no circulant tables, no ADMM or Krylov steps.

Grid convention (Sec. 6.1, generalised to independent axis sizes):
    x_i = i*hx, i = 1..nx, hx = 1/(nx+1)
    y_j = j*hy, j = 1..ny, hy = 1/(ny+1)
    t_k = k*ht, k = 1..nt, ht = T/nt
Fields are float64 arrays of shape (nt, ny, nx): x fastest, time outermost.

The paper evaluates on an analytic target (Sec. 6.1) and uses no dataset; the
workloads below are synthetic in the same spirit.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BASE_SEED = 20191907
INF = math.inf


@dataclasses.dataclass
class Workload:
    """One problem instance: discretisation, data fields and ADMM settings."""

    name: str
    nx: int
    ny: int
    nt: int
    alpha: float  # fractional order along x, in (1, 2]
    beta: float  # fractional order along y, in (1, 2]
    gamma: float  # control regularisation, J2 = gamma * J1
    ua: float
    ub: float
    ya: float = -INF
    yb: float = INF
    T: float = 1.0
    ctrl_sign: float = 1.0  # +1: D y + u = g ; -1: D y - u = g
    delta: float = 1.0
    rho: float = 1.0
    krylov_tol: float = 1e-10
    krylov_maxit: int = 1000
    admm_tol: float = 1e-6
    admm_maxit: int = 100000
    psi_scaling: int = 1  # 1: B and the u copies scaled by psi; 2: B only; 0: none
    obj_weights: int = 0  # 0: all ones, 1: trapezoidal in time (eq. 4.10)
    alpha_t: float = 1.0  # order of the time derivative in (0, 1]; 1 = implicit Euler
    tol_mode: int = 0  # 0: fixed Krylov tolerance; 1: the dynamic rule of Sec. 6.1
    pcg_cold_start: int = 0  # 0: PCG starts from the previous y; 1: from zero
    prox: int = 0  # 0: Algorithm 1; 1: generalized ADMM (Algorithm 2), R_y = c_y I - J1, R_u = c_u I - J2
    prox_cy: float = 0.0  # c_y (0: the smallest admissible, max diag J1)
    prox_cu: float = 0.0  # c_u (0: the smallest admissible, max diag J2)
    precond_kind: int = 0  # 0: S~ of eq. (3.10); 1: the matching approximation S^ of eq. (3.11);
    #                        2: S~ with the diagonal scaling Delta S~^{-1} Delta (variable coefficients)
    krylov_solver: int = 0  # 0: PCG on the normal equations; 1: MINRES on the merged system with K~
    yhat: Optional[np.ndarray] = None  # (nt, ny, nx)
    dplus: Optional[np.ndarray] = None  # (ny, nx) or None (= 1)
    dminus: Optional[np.ndarray] = None  # (ny, nx) or None (= 1)
    g: Optional[np.ndarray] = None  # (nt, ny, nx) or None (= 0)

    @property
    def shape(self):
        return (self.nt, self.ny, self.nx)

    @property
    def N(self):
        return self.nx * self.ny * self.nt

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# ----------------------------------------------------------------------------
# grid coordinates
# ----------------------------------------------------------------------------
def coords(nx: int, ny: int, nt: int, T: float = 1.0):
    """Node coordinates (x_i, y_j, t_k) of the interior space-time grid."""
    x = np.arange(1, nx + 1, dtype=np.float64) / (nx + 1)
    y = np.arange(1, ny + 1, dtype=np.float64) / (ny + 1)
    t = np.arange(1, nt + 1, dtype=np.float64) * (T / nt)
    return x, y, t


def _mesh(nx, ny, nt, T=1.0):
    x, y, t = coords(nx, ny, nt, T)
    return t[:, None, None], y[None, :, None], x[None, None, :]


# ----------------------------------------------------------------------------
# target generators
# ----------------------------------------------------------------------------
def target_sine(nx, ny, nt, T=1.0):
    """yhat = t * sin(pi x) sin(pi y)."""
    t, y, x = _mesh(nx, ny, nt, T)
    return np.ascontiguousarray(t * np.sin(np.pi * x) * np.sin(np.pi * y))


def target_exp_bump(nx, ny, nt, T=1.0):
    """yhat = 16 exp(t) x(1-x) y(1-y)."""
    t, y, x = _mesh(nx, ny, nt, T)
    return np.ascontiguousarray(16.0 * np.exp(t) * x * (1 - x) * y * (1 - y))


def target_paper(nx, ny, nt, T=1.0):
    """The paper's desired state 10 cos(10 x1) sin(x1 x2)(1 - exp(-5t)) (Sec. 6.1)."""
    t, y, x = _mesh(nx, ny, nt, T)
    return np.ascontiguousarray(10 * np.cos(10 * x) * np.sin(x * y) * (1 - np.exp(-5 * t)))


def target_sinusoid_sum(nx, ny, nt, seed, modes=8, T=1.0):
    """yhat = t * sum_m a_m sin(k_m pi x) sin(l_m pi y); a ~ U[0,1], k,l ~ U{1..8}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(0.0, 1.0, size=modes)
    k = rng.integers(1, 9, size=modes)
    l = rng.integers(1, 9, size=modes)
    t, y, x = _mesh(nx, ny, nt, T)
    f = np.zeros((1, ny, nx))
    for m in range(modes):
        f = f + a[m] * np.sin(k[m] * np.pi * x) * np.sin(l[m] * np.pi * y)
    return np.ascontiguousarray(t * f)


def _gauss_smoother(coord: np.ndarray, ell: float, h: float, rng_extent: float):
    """Dense matrix K[i, m] = exp(-(coord_i - s_m)^2 / ell^2) on a noise grid
    s_m of spacing h extending rng_extent beyond [coord.min, coord.max]."""
    lo = coord[0] - rng_extent
    hi = coord[-1] + rng_extent
    m = int(math.ceil((hi - lo) / h)) + 1
    s = lo + h * np.arange(m)
    K = np.exp(-((coord[:, None] - s[None, :]) ** 2) / ell**2)
    return K


def target_grf(nx, ny, nt, seed, ell=0.1, T=1.0):
    """Seeded stationary Gaussian random field on the space-time grid.

    Squared-exponential covariance exp(-|r|^2 / (2 ell^2)) with the same length
    scale on x, y and t.  Built by smoothing white noise with a separable
    Gaussian kernel exp(-s^2/ell^2) on an extended grid (the convolution of
    two such kernels is the required covariance), then normalised to zero
    mean and unit sample variance.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y, t = coords(nx, ny, nt, T)
    ext = 4.0 * ell
    # white noise on a grid of spacing ell/4 (8 samples per kernel width),
    # independent of the output resolution
    hs = ell / 4
    Kx = _gauss_smoother(x, ell, hs, ext)
    Ky = _gauss_smoother(y, ell, hs, ext)
    Kt = _gauss_smoother(t, ell, hs, ext)
    W = rng.standard_normal((Kt.shape[1], Ky.shape[1], Kx.shape[1]))
    F = np.tensordot(Kt, W, axes=([1], [0]))  # (nt, my, mx)
    F = np.einsum("jm,tmx->tjx", Ky, F, optimize=True)  # (nt, ny, mx)
    F = F @ Kx.T  # (nt, ny, nx)
    F = F - F.mean()
    F = F / F.std()
    return np.ascontiguousarray(F)


def coef_sine_x(nx, ny, amp=0.5):
    """d(x, y) = 1 + amp * sin(2 pi x), sampled at interior nodes, shape (ny, nx)."""
    x, y, _ = coords(nx, ny, 1)
    return np.ascontiguousarray(np.broadcast_to(1.0 + amp * np.sin(2 * np.pi * x)[None, :], (ny, nx)).copy())


# ----------------------------------------------------------------------------
# the five workload families
# ----------------------------------------------------------------------------
def small(**kw) -> Workload:
    """16^2 x 8 plain FP64 case (orders 1.5/1.3, box -1 <= u <= 1)."""
    nx, ny, nt = kw.pop("nx", 16), kw.pop("ny", 16), kw.pop("nt", 8)
    w = Workload(name="small_16x16x8", nx=nx, ny=ny, nt=nt, alpha=1.5, beta=1.3,
                 gamma=1e-4, ua=-1.0, ub=1.0)
    w.yhat = target_sine(nx, ny, nt)
    return w.replace(**kw)


def small_mixed(**kw) -> Workload:
    """The small case with box [-5, 5] on u: part of the controls active."""
    return small(ua=-5.0, ub=5.0, name="small_mixed", **kw)


def small_state(**kw) -> Workload:
    """The small case with an active state bound y <= 0.1 and u in [-5, 5]."""
    return small(ua=-5.0, ub=5.0, yb=0.1, name="small_state", **kw)


def headline(nx=256, ny=256, nt=64, ctrl_sign=-1.0, **kw) -> Workload:
    """256^2 x 64, orders 1.3/1.7, d+ = 1 + 0.5 sin(2 pi x), d- = 1,
    yhat = 16 e^t x(1-x) y(1-y), gamma 1e-6, 0 <= u <= 2, y <= 0.8.

    With the control entering as D y + u = g the optimum is exactly zero (the
    operator is an M-matrix), so the meaningful workload takes the control as
    a source (ctrl_sign = -1); ctrl_sign = +1 is the exact-zero check.
    """
    w = Workload(name=f"headline_{nx}x{ny}x{nt}", nx=nx, ny=ny, nt=nt, alpha=1.3, beta=1.7,
                 gamma=1e-6, ua=0.0, ub=2.0, yb=0.8, ctrl_sign=ctrl_sign)
    w.yhat = target_exp_bump(nx, ny, nt)
    w.dplus = coef_sine_x(nx, ny)
    w.dminus = None
    return w.replace(**kw)


def precision(nx=1024, ny=1024, nt=32, **kw) -> Workload:
    """1024^2 x 32, orders 1.8/1.2, GRF target, gamma 1e-5, |u| <= 0.5."""
    w = Workload(name=f"precision_{nx}x{ny}x{nt}", nx=nx, ny=ny, nt=nt, alpha=1.8, beta=1.2,
                 gamma=1e-5, ua=-0.5, ub=0.5)
    w.yhat = target_grf(nx, ny, nt, BASE_SEED + 2)
    return w.replace(**kw)


def differentiation(nx=512, ny=512, nt=32, **kw) -> Workload:
    """512^2 x 32, orders 1.4/1.6, sinusoid-sum target, gamma 1e-4, |u| <= 1."""
    w = Workload(name=f"differentiation_{nx}x{ny}x{nt}", nx=nx, ny=ny, nt=nt, alpha=1.4,
                 beta=1.6, gamma=1e-4, ua=-1.0, ub=1.0)
    w.yhat = target_sinusoid_sum(nx, ny, nt, BASE_SEED + 3)
    return w.replace(**kw)


def paper_test(n=16, alpha_t=0.7, beta=1.3, gamma=1e-4, ya=-4.0, ua=-350.0, delta=2.0, **kw) -> Workload:
    """The paper's test problem (Sec. 6.1): n x n x n grid on (0,1)^2 x (0,T],
    h_t = h_x = 1/(n+1) (so T = n/(n+1)), Caputo time derivative of order
    alpha_t, Riesz derivatives of order beta in both space directions with
    constant coefficients, yhat = 10 cos(10 x1) sin(x1 x2)(1 - exp(-5t)),
    trapezoidal objective weights, symmetric bounds y_b = -y_a and
    u_b = -u_a, D y + u = 0, rho = 1.618, ADMM tolerance 1e-4, the dynamic
    Krylov tolerance, and PCG started from zero in every x-step.  Table 5 of
    the paper pairs n with delta."""
    T = n / (n + 1.0)
    w = Workload(name=f"paper_{n}^3", nx=n, ny=n, nt=n, alpha=beta, beta=beta, gamma=gamma,
                 ua=ua, ub=-ua, ya=ya, yb=-ya, T=T, ctrl_sign=1.0, delta=delta, rho=1.618,
                 admm_tol=1e-4, obj_weights=1, alpha_t=alpha_t, tol_mode=1, pcg_cold_start=1)
    w.yhat = target_paper(n, n, n, T)
    return w.replace(**kw)


BATCH_SIZES = (64, 96, 128, 192, 256, 384, 512)


def batched(count=64, seed=BASE_SEED + 4, sizes=BATCH_SIZES, nts=(16, 32),
            target_seed=BASE_SEED + 4) -> List[Workload]:
    """Uneven instances: nx, ny from `sizes`, nt from `nts`, orders ~ U[1.1, 1.9],
    log10 gamma ~ U[-6, -3], GRF target (seed target_seed+i), |u| <= 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        nx = int(rng.choice(sizes))
        ny = int(rng.choice(sizes))
        nt = int(rng.choice(nts))
        a = float(rng.uniform(1.1, 1.9))
        b = float(rng.uniform(1.1, 1.9))
        gamma = float(10 ** rng.uniform(-6, -3))
        w = Workload(name=f"batch{i}_{nx}x{ny}x{nt}", nx=nx, ny=ny, nt=nt, alpha=a, beta=b,
                     gamma=gamma, ua=-1.0, ub=1.0)
        w.yhat = target_grf(nx, ny, nt, target_seed + i)
        out.append(w)
    return out


BATCH_SMALL_SIZES = (16, 24, 32, 48, 64)


def batched_small(count=256) -> List[Workload]:
    """Many small uneven instances, drawn as in batched(): 16 .. 64 nodes per
    axis, nt 8 or 16 (single launches of such grids cannot fill the GPU)."""
    return batched(count=count, seed=BASE_SEED + 5, sizes=BATCH_SMALL_SIZES, nts=(8, 16),
                   target_seed=BASE_SEED + 1000)


def random_field(shape, seed):
    """Seeded N(0, 1) field (used for operator-apply parity inputs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape)
