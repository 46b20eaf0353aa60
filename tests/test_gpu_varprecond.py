"""The diagonally scaled preconditioner Delta S~^{-1} Delta (precond_kind 2,
variable coefficients) on the GPU against the oracle: the preconditioner
apply (FP64 and FP32 spectrum), the PCG x-step, ADMM iterates, and the
Krylov counts it saves at high coefficient contrast."""
import numpy as np
import pytest

import workloads as W
from oracle import admm
from oracle import operator as op
from oracle import precond as pc
from tests.gpu_util import banner, dev, host, rel, zeros
from tests.test_gpu_parity import make

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1907_13428_amd import fde  # noqa: E402

CASES = ["headline_24x16x8", "ragged_var_24x48x6", "radix3_192x96x12", "min_4x4x4", "radix5_var_50x80x100"]


def scaled(kind):
    w = make(kind).replace(precond_kind=2)
    if kind == "headline_24x16x8":
        w.dplus = W.coef_sine_x(w.nx, w.ny, amp=0.9)
    return w


def oracle_delta(w):
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    return d, sc, pc.scaling_factor(pc.diag_S(w, d, sc.My, sc.Mp, sc.psi))


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("kind", CASES)
def test_scaled_precond_apply(kind, fp32):
    banner("scaled precond", kind, fp32)
    w = scaled(kind).replace(rho=1.2, delta=0.5)
    d, sc, delta = oracle_delta(w)
    tab = pc.precond_tables(w, d)
    r = W.random_field(w.shape, 31)
    ref = pc.apply_precond_scaled(tab, delta, r)
    prob, prm = fde.from_workload(w, precond_fp32=fp32)
    with fde.Context(prob, prm) as ctx:
        z = zeros(w.shape)
        ctx.precond(dev(r), z)
        got = host(z)
    tol = 2e-5 if fp32 else 1e-11
    assert rel(got, ref) <= tol, rel(got, ref)
    np.testing.assert_array_less(np.abs(got - ref), (50 * tol) * np.abs(ref).max())


@pytest.mark.parametrize("kind", ["headline_24x16x8", "radix3_192x96x12", "radix5_var_50x80x100"])
def test_scaled_krylov(kind):
    banner("scaled krylov", kind)
    w = scaled(kind)
    d, sc, delta = oracle_delta(w)
    tab = pc.precond_tables(w, d)
    b = W.random_field(w.shape, 8)
    x0 = 0.1 * W.random_field(w.shape, 9)
    xr, itr, _, ok = admm.pcg(lambda v: admm.apply_S(d, sc, v), lambda v: pc.apply_precond_scaled(tab, delta, v),
                              b, x0, w.krylov_tol, w.krylov_maxit)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        x = dev(x0)
        it, relres, st = ctx.krylov(dev(b), x)
        got = host(x)
    assert st == fde.FDE_OK and ok
    assert abs(it - itr) <= 1, (it, itr)
    assert relres <= w.krylov_tol
    assert rel(got, xr) <= 1e-9, rel(got, xr)


def test_scaled_admm_against_oracle_and_fewer_krylov_iterations():
    """ADMM with the scaled preconditioner follows the oracle's run with it, and
    at d+ = 1 + 0.9 sin 2 pi x takes fewer Krylov iterations than S~."""
    banner("scaled admm")
    w = W.headline(nx=48, ny=32, nt=8).replace(admm_tol=0.0, admm_maxit=6)
    w.dplus = W.coef_sine_x(48, 32, amp=0.9)
    counts = {}
    for kind in (0, 2):
        wk = w.replace(precond_kind=kind)
        ref = admm.admm_solve(wk, iters=6)
        prob, prm = fde.from_workload(wk)
        with fde.Context(prob, prm) as ctx:
            state, st, _ = ctx.admm_solve(dev(wk.yhat))
            got = {k: host(v) for k, v in state.items()}
        for k in ("y", "u", "p"):
            assert rel(got[k], getattr(ref, k)) <= 1e-7, (kind, k, rel(got[k], getattr(ref, k)))
        assert abs(st["pcg_total"] - sum(ref.pcg_iters)) <= 6, (st["pcg_total"], ref.pcg_iters)
        counts[kind] = st["pcg_total"]
    assert counts[2] < counts[0], counts


def test_scaled_precond_rejected_with_minres():
    banner("scaled precond with MINRES")
    w = scaled("headline_24x16x8").replace(krylov_solver=1)
    prob, prm = fde.from_workload(w)
    with pytest.raises(fde.FdeError) as e:
        fde.Context(prob, prm)
    assert e.value.status == fde.FDE_EINVAL
