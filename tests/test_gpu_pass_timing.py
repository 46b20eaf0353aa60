"""In-solve pass timing (fde_pass_timing / fde_pass_stats): with events bound
to each pass launch, the PCG iterations run as plain launches and must give
the graph launches' results bit for bit; every one of the nine passes is timed
once per PCG iteration enqueued."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import banner, dev, host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1907_13428_amd import fde  # noqa: E402


def test_pass_timing_leaves_results_unchanged():
    banner("pass timing", "headline 48x32x8")
    w = W.headline(nx=48, ny=32, nt=8).replace(admm_tol=0.0, admm_maxit=15)
    prob, prm = fde.from_workload(w)
    yhat = dev(w.yhat)
    out = []
    for timed in (False, True):
        with fde.Context(prob, prm) as ctx:
            if timed:
                ctx.pass_timing(True)
            state, st, _ = ctx.admm_solve(yhat)
            out.append(({k: host(v) for k, v in state.items()}, st))
            if timed:
                ps = ctx.pass_stats()
                ctx.pass_timing(False)
    (a, sa), (b, sb) = out
    assert sa["pcg_total"] == sb["pcg_total"] and sa["admm_iters"] == sb["admm_iters"]
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    counts = {n for _, n, _ in ps.values()}
    assert len(counts) == 1 and counts.pop() >= sb["pcg_total"]
    for name, (us, n, by) in ps.items():
        assert us > 0 and by > 0, name


def test_pass_timing_rejects_fractional_time():
    banner("pass timing", "Caputo rejected")
    w = W.small(nx=16, ny=16, nt=8).replace(alpha_t=0.7)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        with pytest.raises(fde.FdeError) as e:
            ctx.pass_timing(True)
        assert e.value.status == fde.FDE_EINVAL
