"""fde_set_params on a live context: the new ADMM settings (gamma, delta, rho,
Algorithm 2, the matching preconditioner of eq. (3.11), the diagonally scaled
S~ of variable coefficients) must reach every
kernel of the next solve, including the PCG iterations replayed from the
captured graph, whose launches hold the preconditioner's scalars by value.

Each case first solves with the initial settings (which captures the graph on
the same solution buffer), switches the settings, solves again on the same
buffers, and compares bitwise with a fresh context created with the new
settings, and with the oracle (PCG count +-1, solution 1e-9; ADMM count and
iterates as in the parity tests).
"""
import numpy as np
import pytest

import workloads as W
from oracle import admm
from oracle import operator as op
from oracle import precond as pc
from tests.gpu_util import banner, dev, host, rel, zeros

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1907_13428_amd import fde  # noqa: E402

CHANGES = {
    "rho_gamma_delta": dict(rho=1.5, gamma=1e-3, delta=0.4),
    "matching_precond": dict(precond_kind=1),
    "alg2": dict(prox=1, rho=0.8, prox_cy=1.5, prox_cu=2e-6),
    "scaled_precond": dict(precond_kind=2, rho=1.2),
}


def _base():
    return W.headline(nx=24, ny=16, nt=8)


@pytest.mark.parametrize("name", list(CHANGES))
def test_set_params_krylov_uses_new_preconditioner(name):
    banner("set_params krylov", name)
    w0 = _base()
    w1 = w0.replace(**CHANGES[name])
    b = W.random_field(w0.shape, 8)
    x0 = 0.1 * W.random_field(w0.shape, 9)
    prob, prm0 = fde.from_workload(w0)
    _, prm1 = fde.from_workload(w1)
    with fde.Context(prob, prm0) as ctx:
        x = dev(x0)
        bd = dev(b)
        ctx.krylov(bd, x)  # captures the PCG graph on x with the old scalars
        x.copy_(dev(x0))
        ctx.set_params(prm1)
        it, relres, st = ctx.krylov(bd, x)
        got = host(x)
    with fde.Context(prob, prm1) as fresh:
        xf = dev(x0)
        itf, _, stf = fresh.krylov(dev(b), xf)
        want = host(xf)
    assert st == fde.FDE_OK and stf == fde.FDE_OK
    assert it == itf and np.array_equal(got, want), (it, itf)
    d = op.disc_from(w1)
    sc = admm.scalars(w1, d)
    tab = pc.precond_tables(w1, d)
    if w1.precond_kind == 2:
        delta = pc.scaling_factor(pc.diag_S(w1, d, sc.My, sc.Mp, sc.psi))
        M = lambda v: pc.apply_precond_scaled(tab, delta, v)
    else:
        M = lambda v: pc.apply_precond(tab, v)
    xr, itr, _, ok = admm.pcg(lambda v: admm.apply_S(d, sc, v), M, b, x0, w1.krylov_tol, w1.krylov_maxit)
    assert ok and abs(it - itr) <= 1, (it, itr)
    assert relres <= w1.krylov_tol
    assert rel(got, xr) <= 1e-9, rel(got, xr)


@pytest.mark.parametrize("name", list(CHANGES))
def test_set_params_admm_uses_new_settings(name):
    banner("set_params admm", name)
    K = 12
    w0 = _base().replace(admm_tol=0.0, admm_maxit=K)
    w1 = w0.replace(**CHANGES[name])
    prob, prm0 = fde.from_workload(w0)
    _, prm1 = fde.from_workload(w1)
    yhat = dev(w0.yhat)
    with fde.Context(prob, prm0) as ctx:
        state, _, _ = ctx.admm_solve(yhat)
        for t in state.values():
            t.zero_()
        ctx.set_params(prm1)
        state, stats, _ = ctx.admm_solve(yhat, state=state)
        got = {k: host(v) for k, v in state.items()}
    with fde.Context(prob, prm1) as fresh:
        sf, statsf, _ = fresh.admm_solve(yhat)
        want = {k: host(v) for k, v in sf.items()}
    assert stats["admm_iters"] == statsf["admm_iters"] == K
    assert stats["pcg_total"] == statsf["pcg_total"]
    for k in want:
        assert np.array_equal(got[k], want[k]), k
    ref = admm.admm_solve(w1, iters=K)
    for k in ("y", "u", "p"):
        r = getattr(ref, k)
        assert rel(got[k], r) <= 1e-7, (k, rel(got[k], r))
