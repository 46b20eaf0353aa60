"""GPU: the adjoint (transposed-Toeplitz) solve and the gradients of the optimal
value, against the oracle (sparse LU adjoint, polished optima, central differences)."""
import numpy as np
import pytest

import workloads as W
from oracle import admm, grad, kkt
from oracle import operator as op
from tests.gpu_util import banner, dev, host, rel, zeros

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1907_13428_amd import fde  # noqa: E402


def var_problem(nx=12, ny=8, nt=6):
    w = W.small_mixed(nx=nx, ny=ny, nt=nt).replace(alpha=1.4, beta=1.6)
    w.yhat = 3.0 * W.target_sinusoid_sum(nx, ny, nt, W.BASE_SEED + 3)
    w.dplus = W.coef_sine_x(nx, ny)
    return w


@pytest.mark.parametrize("var", [False, True])
@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("alpha_t", [1.0, 0.6])
def test_adjoint_solve_matches_sparse_lu(var, fp32, alpha_t):
    """Backward time stepping of D^T lambda = f against a sparse LU of D^T; with
    a Caputo order the history of later time levels enters every step."""
    banner("adjoint solve", var, fp32, alpha_t)
    w = var_problem().replace(alpha_t=alpha_t)
    if not var:
        w.dplus = None
    rng = np.random.Generator(np.random.PCG64(11))
    y = rng.standard_normal(w.shape)
    wy = rng.standard_normal(w.shape)
    ref = grad.adjoint_multiplier(w, y, wy)
    prob, prm = fde.from_workload(w, precond_fp32=fp32)
    with fde.Context(prob, prm) as ctx:
        lam = zeros(w.shape)
        ctx.grad(dev(w.yhat), dev(y), zeros(w.shape), dev(wy), adjoint_solve=True, lam=lam)
        got = host(lam)
    assert rel(got, ref) <= 1e-10, rel(got, ref)


def test_adjoint_grad_on_polished_optimum_matches_oracle_and_fd():
    banner("adjoint gradients on the polished optimum")
    w = var_problem()
    r = admm.admm_solve(w.replace(admm_tol=1e-9))
    pol = kkt.polish(w, r.zy, r.zu)
    assert pol["ok"]
    gy, ga, gb = grad.gradients(w, pol["y"], pol["lam"])
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        dy = zeros(w.shape)
        lam = zeros(w.shape)
        _, da, db = ctx.grad(dev(w.yhat), dev(pol["y"]), zeros(w.shape), dev(pol["mu_y"]), adjoint_solve=True,
                             dyhat=dy, lam=lam)
        dyh, lamg = host(dy), host(lam)
    assert rel(lamg, pol["lam"]) <= 1e-9
    assert rel(dyh, gy) <= 1e-14
    assert abs(da - ga) <= 1e-9 * abs(ga) and abs(db - gb) <= 1e-9 * abs(gb)
    # central differences of the exact optimal value (same active set at +-h)
    h = 1e-6
    for name, g in (("alpha", da), ("beta", db)):
        a0 = getattr(w, name)
        jp = kkt.polish(w.replace(**{name: a0 + h}), r.zy, r.zu)
        jm = kkt.polish(w.replace(**{name: a0 - h}), r.zy, r.zu)
        fd = (jp["J"] - jm["J"]) / (2 * h)
        assert abs(fd - g) <= 1e-6 * max(abs(g), 1e-3), (name, fd, g)


def test_differentiation_workload_gradients_32x32x8():
    """The differentiation workload at 32^2 x 8: GPU ADMM solve, GPU adjoint
    gradients, against central differences (h = 1e-6) of the exact optimal
    value on the GPU solution's active set."""
    banner("differentiation 32x32x8")
    w = W.differentiation(nx=32, ny=32, nt=8).replace(admm_tol=1e-9, admm_maxit=60000)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        state, stats, status = ctx.admm_solve(dev(w.yhat))
        assert status == fde.FDE_OK, stats
        dy = zeros(w.shape)
        _, da, db = ctx.grad(dev(w.yhat), state["y"], state["p"], state["wy"], adjoint_solve=True, dyhat=dy)
        zy, zu, yg = host(state["zy"]), host(state["zu"]), host(state["y"])
        dyh = host(dy)
    pol = kkt.polish(w, zy, zu)
    assert pol["ok"]
    h = 1e-6
    for name, g in (("alpha", da), ("beta", db)):
        a0 = getattr(w, name)
        fd = (kkt.polish(w.replace(**{name: a0 + h}), zy, zu)["J"]
              - kkt.polish(w.replace(**{name: a0 - h}), zy, zu)["J"]) / (2 * h)
        assert abs(fd - g) <= 1e-5 * abs(fd), (name, fd, g)
    # dJ/dyhat at a few entries: central differences of the exact optimal value
    gy_exact = -(pol["y"] - w.yhat)
    assert rel(dyh, gy_exact) <= 1e-4
    rng = np.random.Generator(np.random.PCG64(2))
    for _ in range(2):
        idx = tuple(int(rng.integers(0, s)) for s in w.shape)
        wp, wm = w.replace(yhat=w.yhat.copy()), w.replace(yhat=w.yhat.copy())
        wp.yhat[idx] += h
        wm.yhat[idx] -= h
        fd = (kkt.polish(wp, zy, zu)["J"] - kkt.polish(wm, zy, zu)["J"]) / (2 * h)
        assert abs(fd - gy_exact[idx]) <= 1e-6 * max(1.0, abs(fd))
        assert abs(fd - dyh[idx]) <= 1e-4 * max(1.0, abs(fd))


def test_autograd_function():
    banner("autograd")
    from paper_1907_13428_amd.autograd import objective, spec_from_workload

    w = var_problem().replace(admm_tol=1e-9, admm_maxit=60000)
    yhat = dev(w.yhat).requires_grad_(True)
    a = torch.tensor(w.alpha, dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.tensor(w.beta, dtype=torch.float64, device="cuda", requires_grad=True)
    J = objective(yhat, a, b, **spec_from_workload(w))
    J.backward()
    r = admm.admm_solve(w)
    pol = kkt.polish(w, r.zy, r.zu)
    gy, ga, gb = grad.gradients(w, pol["y"], pol["lam"])
    assert abs(J.item() - pol["J"]) <= 1e-6 * abs(pol["J"])
    assert rel(host(yhat.grad), gy) <= 1e-5
    assert abs(a.grad.item() - ga) <= 1e-5 * abs(ga)
    assert abs(b.grad.item() - gb) <= 1e-5 * abs(gb)
