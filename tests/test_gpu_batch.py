"""GPU: the batched form (uneven instances driven concurrently)."""
import numpy as np
import pytest

import workloads as W
from oracle import admm
from tests.gpu_util import banner, dev, host, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1907_13428_amd import fde  # noqa: E402


def uneven(count=6, seed=5):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        nx, ny = int(rng.choice([8, 12, 16, 24])), int(rng.choice([8, 12, 16]))
        nt = int(rng.choice([4, 6, 8]))
        w = W.small_mixed(nx=nx, ny=ny, nt=nt).replace(alpha=float(rng.uniform(1.1, 1.9)),
                                                       beta=float(rng.uniform(1.1, 1.9)),
                                                       gamma=float(10 ** rng.uniform(-5, -3)))
        w.yhat = W.target_grf(nx, ny, nt, W.BASE_SEED + 100 + i)
        out.append(w)
    return out


def run(ws, concurrent, fp32=0):
    probs, prms = zip(*[fde.from_workload(w, precond_fp32=fp32) for w in ws])
    with fde.Batch(list(probs), list(prms)) as b:
        states, stats, codes = b.solve([dev(w.yhat) for w in ws], concurrent=concurrent)
        return [{k: host(v) for k, v in s.items()} for s in states], stats, codes


def test_batch_concurrent_equals_sequential_and_oracle():
    banner("batch concurrent vs sequential")
    ws = uneven()
    a, sa, ca = run(ws, True)
    b, sb, cb = run(ws, False)
    assert ca == cb
    for i in range(len(ws)):
        assert sa[i]["admm_iters"] == sb[i]["admm_iters"]
        for k in a[i]:
            assert np.array_equal(a[i][k], b[i][k]), (i, k)
    for i in (0, 3):
        w = ws[i]
        K = sa[i]["admm_iters"]
        ref = admm.admm_solve(w, iters=K)
        assert rel(a[i]["y"], ref.y) <= 1e-7 and rel(a[i]["u"], ref.u) <= 1e-7


def test_batch_fp32_preconditioner_error_stated():
    banner("batch fp32 precond")
    ws = uneven(count=3, seed=8)
    a, sa, _ = run(ws, True, fp32=1)
    for i, w in enumerate(ws):
        ref = admm.admm_solve(w, iters=sa[i]["admm_iters"])
        assert rel(a[i]["y"], ref.y) <= 1e-7, i


def test_batch_rejects_invalid_instance():
    banner("batch invalid")
    ws = uneven(count=2)
    probs, prms = zip(*[fde.from_workload(w) for w in ws])
    probs = list(probs)
    probs[1].nx = 10
    with pytest.raises(fde.FdeError) as e:
        fde.Batch(probs, list(prms))
    assert "instance 1" in str(e.value)


def test_batch_mixed_methods_concurrent_equals_sequential_and_oracle():
    """Instances that each pick a different method (Algorithm 2, the matching
    preconditioner, the MINRES x-step, a Caputo time order) run together:
    concurrent and sequential runs agree bitwise, and every instance follows
    the oracle."""
    banner("batch mixed methods")
    ws = uneven(count=4, seed=11)
    ws[0] = ws[0].replace(prox=1, prox_cy=1.5, rho=0.9)
    ws[1] = ws[1].replace(precond_kind=1)
    ws[2] = ws[2].replace(krylov_solver=1)
    ws[3] = ws[3].replace(alpha_t=0.6, krylov_solver=1, prox=1)
    ws = [w.replace(admm_tol=0.0, admm_maxit=20) for w in ws]
    a, sa, ca = run(ws, True)
    b, sb, cb = run(ws, False)
    assert ca == cb
    for i in range(len(ws)):
        assert sa[i]["admm_iters"] == sb[i]["admm_iters"] == 20
        assert sa[i]["pcg_total"] == sb[i]["pcg_total"]
        for k in a[i]:
            assert np.array_equal(a[i][k], b[i][k]), (i, k)
    for i, w in enumerate(ws):
        ref = admm.admm_solve(w, iters=20)
        assert abs(sa[i]["pcg_total"] - sum(ref.pcg_iters)) <= 20, (i, sa[i]["pcg_total"], sum(ref.pcg_iters))
        for k in ("y", "u", "p", "wy", "wu"):
            assert rel(a[i][k], getattr(ref, k)) <= 1e-7, (i, k)


def batchable(count=4, seed=21, maxit=None, sizes=(64, 96, 128), nts=(16, 32)):
    """Uneven instances on lengths with batched passes (by default 64, 96, 128
    nodes in space; 16 and 32 time levels)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        nx, ny = int(rng.choice(sizes)), int(rng.choice(sizes))
        nt = int(rng.choice(nts))
        w = W.small_mixed(nx=nx, ny=ny, nt=nt).replace(alpha=float(rng.uniform(1.1, 1.9)),
                                                       beta=float(rng.uniform(1.1, 1.9)),
                                                       gamma=float(10 ** rng.uniform(-5, -3)))
        w.yhat = W.target_grf(nx, ny, nt, W.BASE_SEED + 200 + i)
        if maxit is not None:
            w = w.replace(admm_tol=0.0, admm_maxit=maxit + 3 * i)
        out.append(w)
    return out


def run_mode(ws, mode, fp32=0):
    probs, prms = zip(*[fde.from_workload(w, precond_fp32=fp32) for w in ws])
    with fde.Batch(list(probs), list(prms)) as b:
        states, stats, codes = b.solve([dev(w.yhat) for w in ws], concurrent=(mode != "sequential"),
                                       lockstep=(mode == "lockstep"))
        return [{k: host(v) for k, v in s.items()} for s in states], stats, codes


def max_rel(a, b):
    nb = float(np.max(np.abs(b)))
    return float(np.max(np.abs(a - b))) / (nb if nb > 0 else 1.0)


# The batched pass kernels run the single kernels' code, with each instance's
# arguments read from a table into the block's own copy and that instance's
# block decomposition: the lockstep run equals the per-instance solves bit for
# bit, FP64 and FP32 preconditioner alike.
@pytest.mark.parametrize("fp32", [0, 1])
def test_batch_lockstep_equals_sequential_and_oracle(fp32):
    """Lockstep mode (the Krylov iterations of all instances as batched pass
    launches): uneven instances with different ADMM budgets take the same
    Krylov and ADMM iteration counts as the per-instance solves and the same
    iterates bit for bit, and follow the oracle."""
    banner("batch lockstep vs sequential", fp32)
    ws = batchable(maxit=6)
    a, sa, ca = run_mode(ws, "lockstep", fp32)
    b, sb, cb = run_mode(ws, "sequential", fp32)
    assert ca == cb
    assert all(s["batched"] == 1 for s in sa) and all(s["batched"] == 0 for s in sb)
    for i in range(len(ws)):
        assert sa[i]["admm_iters"] == sb[i]["admm_iters"] == ws[i].admm_maxit
        assert sa[i]["pcg_total"] == sb[i]["pcg_total"]
        for k in a[i]:
            assert np.array_equal(a[i][k], b[i][k]), (i, k, max_rel(a[i][k], b[i][k]))
    for i in (0, 3):
        ref = admm.admm_solve(ws[i], iters=ws[i].admm_maxit)
        for k in ("y", "u", "p"):
            assert rel(a[i][k], getattr(ref, k)) <= 1e-7, (i, k)


def test_batch_lockstep_small_instances():
    """Many small uneven grids (16 .. 48 nodes in space, 8 and 16 time levels,
    the regime where single launches cannot fill the GPU): the lockstep run
    equals the per-instance solves bit for bit."""
    banner("batch lockstep small instances")
    ws = batchable(count=12, seed=33, maxit=4, sizes=(16, 24, 32, 48), nts=(8, 16))
    for i in (1, 4, 7):  # the diagonally scaled preconditioner in some of them
        ws[i] = ws[i].replace(precond_kind=2)
    a, sa, ca = run_mode(ws, "lockstep")
    b, sb, cb = run_mode(ws, "sequential")
    assert ca == cb
    assert all(s["batched"] == 1 for s in sa)
    for i in range(len(ws)):
        assert sa[i]["pcg_total"] == sb[i]["pcg_total"] and sa[i]["admm_iters"] == sb[i]["admm_iters"]
        for k in a[i]:
            assert np.array_equal(a[i][k], b[i][k]), (i, k, max_rel(a[i][k], b[i][k]))


def test_batch_lockstep_converging_instances():
    """Instances that stop at different ADMM iterations on the stopping test:
    the lockstep run keeps the finished ones out and equals the per-instance
    solves."""
    banner("batch lockstep converging")
    # the paper's test problem on 64^3 with implicit Euler in time, three box settings
    ws = [W.paper_test(64, alpha_t=1.0, ya=ya, ua=ua, delta=0.4).replace(admm_maxit=400)
          for ya, ua in ((-7.0, -400.0), (-4.0, -350.0), (-1.0, -400.0))]
    a, sa, ca = run_mode(ws, "lockstep")
    b, sb, cb = run_mode(ws, "sequential")
    assert ca == cb
    assert all(s["batched"] == 1 for s in sa)
    assert len({s["admm_iters"] for s in sb}) > 1  # the instances stop at different iterations
    for i in range(len(ws)):
        assert sa[i]["admm_iters"] == sb[i]["admm_iters"]
        for k in a[i]:
            assert np.array_equal(a[i][k], b[i][k]), (i, k, max_rel(a[i][k], b[i][k]))


def test_batch_lockstep_falls_back_without_batched_passes():
    """Lengths without batched passes (and the MINRES x-step) make the lockstep
    request run the concurrent mode: same results as sequential."""
    banner("batch lockstep fallback")
    ws = uneven(count=3, seed=2)
    ws = [w.replace(admm_tol=0.0, admm_maxit=8) for w in ws]
    a, sa, _ = run_mode(ws, "lockstep")
    b, sb, _ = run_mode(ws, "sequential")
    assert all(s["batched"] == 0 for s in sa)  # the concurrent mode ran
    for i in range(len(ws)):
        for k in a[i]:
            assert np.array_equal(a[i][k], b[i][k]), (i, k)
