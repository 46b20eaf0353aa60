"""GPU: per-point box bounds (fde_set_bounds) against the oracle, and the
checks that guard them."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import admm, kkt
from tests.gpu_util import banner, dev, host, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1907_13428_amd import fde  # noqa: E402

KEYS = ("y", "u", "zy", "zu", "p", "wy", "wu")


def grid(w):
    t = (np.arange(1, w.nt + 1) * (w.T / w.nt))[:, None, None]
    y = (np.arange(1, w.ny + 1) / (w.ny + 1))[None, :, None]
    x = (np.arange(1, w.nx + 1) / (w.nx + 1))[None, None, :]
    return t, y, x


def varying_control(nx=16, ny=12, nt=8):
    w = W.small(nx=nx, ny=ny, nt=nt)
    t, y, x = grid(w)
    ua = -0.2 - 0.5 * x * np.ones(w.shape)
    ub = 0.1 + 0.8 * t * y * np.ones(w.shape)
    ua[0, :, :2] = -np.inf
    return w.replace(ua=ua, ub=ub)


def varying_state(nx=16, ny=12, nt=8):
    w = W.small_state(nx=nx, ny=ny, nt=nt)
    t, y, x = grid(w)
    return w.replace(yb=0.02 + 0.15 * t * (1.0 + x) * np.ones(w.shape))


def solve_gpu(w, scalar_w, arrays):
    """ADMM with the array bounds passed through fde_set_bounds; the scalar
    parameters come from scalar_w (the sides without an array)."""
    prob, prm = fde.from_workload(scalar_w)
    with fde.Context(prob, prm) as ctx:
        ctx.set_bounds(**{k: dev(np.ascontiguousarray(v)) for k, v in arrays.items()})
        state, stats, status = ctx.admm_solve(dev(w.yhat))
        return {k: host(v) for k, v in state.items()}, stats, status


@pytest.mark.parametrize("kind", ["control", "state"])
def test_per_point_bounds_match_oracle(kind):
    banner("per-point bounds", kind)
    if kind == "control":
        w = varying_control()
        scalar_w = w.replace(ua=-math.inf, ub=math.inf)
        arrays = {"ua": w.ua, "ub": w.ub}
    else:
        w = varying_state()
        scalar_w = w.replace(yb=math.inf)
        arrays = {"yb": w.yb}
    got, stats, status = solve_gpu(w, scalar_w, arrays)
    ref = admm.admm_solve(w)
    assert status == fde.FDE_OK and ref.converged
    K = stats["admm_iters"]
    assert abs(K - ref.iters) <= 1
    if K != ref.iters:
        ref = admm.admm_solve(w, iters=K)
    for k in KEYS:
        assert rel(got[k], getattr(ref, k)) <= 1e-7, k
    pol = kkt.polish(w, got["zy"], got["zu"])
    assert pol["ok"]
    ya, yb, ua, ub = (b.reshape(w.shape) for b in kkt.bounds_flat(w))
    assert np.all(got["zy"] >= ya) and np.all(got["zy"] <= yb)
    assert np.all(got["zu"] >= ua) and np.all(got["zu"] <= ub)


def test_constant_arrays_equal_scalar_bounds_and_reset():
    banner("per-point bounds: constant arrays, reset")
    w = W.small_state(nx=12, ny=8, nt=6).replace(admm_tol=0.0, admm_maxit=30)
    prob, prm = fde.from_workload(w)
    yhat = dev(w.yhat)
    with fde.Context(prob, prm) as ctx:
        s0, _, _ = ctx.admm_solve(yhat)
        a = {k: host(v) for k, v in s0.items()}
        full = lambda v: dev(np.full(w.shape, v))
        ctx.set_bounds(ya=full(w.ya), yb=full(w.yb), ua=full(w.ua), ub=full(w.ub))
        s1, _, _ = ctx.admm_solve(yhat)
        b = {k: host(v) for k, v in s1.items()}
        ctx.set_bounds()  # all None: scalar bounds again
        s2, _, _ = ctx.admm_solve(yhat)
        c = {k: host(v) for k, v in s2.items()}
    for k in KEYS:
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k]), k


def test_bound_checks():
    banner("per-point bounds: checks")
    w = W.small(nx=12, ny=8, nt=6)
    prob, prm = fde.from_workload(w)  # scalar box -1 <= u <= 1
    with fde.Context(prob, prm) as ctx:
        lo = np.full(w.shape, -0.5)
        lo[2, 3, 4] = 2.0  # above the scalar upper bound 1
        with pytest.raises(fde.FdeError) as e:
            ctx.set_bounds(ua=dev(lo))
        assert e.value.status == fde.FDE_EINVAL and "lower bound" in str(e.value)
        bad = np.full(w.shape, 0.5)
        bad[0, 0, 0] = np.nan
        with pytest.raises(fde.FdeError):
            ctx.set_bounds(ub=dev(bad))
        with pytest.raises(ValueError):
            ctx.set_bounds(ua=dev(np.zeros((2, 2, 2))))
        # a valid array, then scalar parameters that contradict it
        ctx.set_bounds(ua=dev(np.full(w.shape, 0.2)))
        with pytest.raises(fde.FdeError):
            ctx.set_params(fde.from_workload(w.replace(ub=0.1))[1])
        ctx.set_params(fde.from_workload(w.replace(ub=0.5))[1])
