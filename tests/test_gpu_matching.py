"""GPU: the matching Schur-complement approximation of eq. (3.11) with circulant
blocks (precond_kind = 1) against the oracle: the preconditioner apply in FP64
and FP32, PCG and ADMM iterates, and the 256^2 x 64 headline grid."""
import numpy as np
import pytest

import workloads as W
from oracle import admm, kkt, precond
from oracle import operator as op
from tests.gpu_util import banner, dev, host, rel, zeros

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1907_13428_amd import fde  # noqa: E402

KEYS = ("y", "u", "zy", "zu", "p", "wy", "wu")


def case(kind):
    if kind == "small":
        return W.small_mixed(precond_kind=1)
    if kind == "var_ragged":
        w = W.small(nx=24, ny=48, nt=6, alpha=1.3, beta=1.7, precond_kind=1)
        w.dplus = W.coef_sine_x(24, 48)
        return w
    if kind == "radix3_prox":
        return W.small(nx=48, ny=24, nt=12, alpha=1.45, beta=1.55, precond_kind=1, prox=1, rho=0.9)
    if kind == "caputo":
        return W.small(nx=16, ny=12, nt=8, alpha_t=0.6, T=0.9, precond_kind=1)
    raise KeyError(kind)


@pytest.mark.parametrize("kind", ["small", "var_ragged", "radix3_prox", "caputo"])
def test_matching_preconditioner_apply(kind):
    banner("matching precond", kind)
    w = case(kind)
    tab = precond.precond_tables(w, op.disc_from(w))
    assert tab["kind"] == 1
    v = W.random_field(w.shape, 51)
    ref = precond.apply_precond(tab, v)
    ref0 = precond.apply_precond(dict(tab, kind=0), v)
    assert rel(ref, ref0) > 1e-3  # a different operator from S~
    for fp32 in (0, 1):
        prob, prm = fde.from_workload(w, precond_fp32=fp32)
        with fde.Context(prob, prm) as ctx:
            y = zeros(w.shape)
            ctx.precond(dev(v), y)
            assert rel(host(y), ref) <= (2e-5 if fp32 else 1e-11), fp32


@pytest.mark.parametrize("kind", ["small", "radix3_prox"])
def test_matching_preconditioner_admm(kind):
    banner("matching precond admm", kind)
    w = case(kind).replace(ua=-5.0, ub=5.0)
    fixed = kind == "radix3_prox"  # converges slowly: compared after a fixed 40 iterations
    if fixed:
        w = w.replace(admm_tol=0.0, admm_maxit=40)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        state, stats, status = ctx.admm_solve(dev(w.yhat))
        got = {k: host(v) for k, v in state.items()}
    ref = admm.admm_solve(w, iters=w.admm_maxit if fixed else None)
    assert status == (fde.FDE_ENOTCONV if fixed else fde.FDE_OK) and (fixed or ref.converged)
    K = stats["admm_iters"]
    assert abs(K - ref.iters) <= 1
    assert abs(stats["pcg_total"] - sum(ref.pcg_iters)) <= K
    if K != ref.iters:
        ref = admm.admm_solve(w, iters=K)
    for k in KEYS:
        assert rel(got[k], getattr(ref, k)) <= 1e-7, k
    if not fixed:
        assert kkt.polish(w, got["zy"], got["zu"])["ok"]


def test_matching_preconditioner_headline_full_size():
    """256^2 x 64 in the benchmark's launch configuration: S^^{-1} v element by
    element, and five PCG iterations from zero with it."""
    banner("full size: matching precond headline")
    w = W.headline(precond_kind=1)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    tab = precond.precond_tables(w, d)
    v = W.random_field(w.shape, 52)
    b = W.random_field(w.shape, 53)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        ctx.autotune()
        y = zeros(w.shape)
        ctx.precond(dev(v), y)
        z = host(y)
        ctx.set_params(fde.from_workload(w, krylov_maxit=5, krylov_tol=1e-30)[1])
        x = zeros(w.shape)
        it, relres, st = ctx.krylov(dev(b), x)
        xg = host(x)
    assert rel(z, precond.apply_precond(tab, v)) <= 1e-12
    xr, itr, relr, conv = admm.pcg(lambda u: admm.apply_S(d, sc, u), lambda u: precond.apply_precond(tab, u), b,
                                   np.zeros(w.shape), 1e-30, 5)
    assert st == fde.FDE_ENOTCONV and it == 5 and itr == 5
    assert rel(xg, xr) <= 1e-10 and abs(relres - relr) <= 1e-8 * relr
