"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars: operator applies 1e-11 relative (2-norm); FP64 preconditioner 1e-11;
FP32 preconditioner 2e-5 (a float32 3-D FFT, error grows like eps32 log N);
PCG solutions 1e-9 at equal iteration counts; ADMM solutions 1e-7 relative
at equal ADMM iteration counts.
"""
import numpy as np
import pytest

import workloads as W
from oracle import admm, kkt
from oracle import operator as op
from oracle import precond as pc
from tests.gpu_util import banner, dev, host, rel, zeros

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1907_13428_amd import fde  # noqa: E402


def var_fields(w, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    w.dplus = W.coef_sine_x(w.nx, w.ny)
    w.dminus = 1.0 + 0.3 * rng.uniform(size=(w.ny, w.nx))
    return w


def make(kind):
    if kind == "small":
        return W.small()
    if kind == "headline_24x16x8":
        return W.headline(nx=24, ny=16, nt=8)
    if kind == "ragged_var_24x48x6":
        return var_fields(W.small(nx=24, ny=48, nt=6).replace(alpha=1.3, beta=1.7))
    if kind == "const_96x12x4":
        return W.small(nx=96, ny=12, nt=4).replace(alpha=1.8, beta=1.2)
    if kind == "tiny_var_6x8x4":
        return var_fields(W.small(nx=6, ny=8, nt=4))
    if kind == "laplace_48x24x6":
        return W.small(nx=48, ny=24, nt=6).replace(alpha=2.0, beta=2.0)
    if kind == "radix3_192x96x12":
        return var_fields(W.small(nx=192, ny=96, nt=12).replace(alpha=1.45, beta=1.55))
    if kind == "long_1024x8x4":
        return W.small(nx=1024, ny=8, nt=4).replace(alpha=1.6, beta=1.4)
    if kind == "tall_8x1024x4":
        return var_fields(W.small(nx=8, ny=1024, nt=4))
    if kind == "min_4x4x4":  # the smallest supported length on every axis
        return var_fields(W.small(nx=4, ny=4, nt=4).replace(alpha=1.7, beta=1.3))
    if kind == "min_mixed_4x6x12":
        return W.small(nx=4, ny=6, nt=12).replace(alpha=1.2, beta=1.9)
    # lengths with a factor 5: radix-5 preconditioner transforms, longer operator embeddings
    if kind == "radix5_var_50x80x100":
        return var_fields(W.small(nx=50, ny=80, nt=100).replace(alpha=1.35, beta=1.65))
    if kind == "radix5_160x100x50":
        return W.small(nx=160, ny=100, nt=50).replace(alpha=1.8, beta=1.2)
    if kind == "radix5_colcoef_100x50x8":
        return W.headline(nx=100, ny=50, nt=8)
    # columns of 1024 points and more: tiles without the spare LDS column
    if kind == "tall_var_8x768x4":  # 1536-point operator columns
        return var_fields(W.small(nx=8, ny=768, nt=4).replace(alpha=1.6, beta=1.3))
    if kind == "tall_6x512x6":  # 1024-point operator columns
        return W.small(nx=6, ny=512, nt=6).replace(alpha=1.25, beta=1.75)
    if kind == "deep_4x6x1024":  # 1024-point preconditioner columns along t
        return W.small(nx=4, ny=6, nt=1024)
    raise KeyError(kind)


OP_CASES = ["small", "headline_24x16x8", "ragged_var_24x48x6", "const_96x12x4", "tiny_var_6x8x4",
            "laplace_48x24x6", "radix3_192x96x12", "long_1024x8x4", "tall_8x1024x4", "min_4x4x4",
            "min_mixed_4x6x12", "radix5_var_50x80x100", "radix5_160x100x50", "radix5_colcoef_100x50x8",
            "tall_var_8x768x4", "tall_6x512x6", "deep_4x6x1024"]


@pytest.fixture(scope="module", autouse=True)
def _built():
    fde.lib()


@pytest.mark.parametrize("kind", OP_CASES)
@pytest.mark.parametrize("transpose", [False, True])
def test_apply_A(kind, transpose):
    banner("apply_A", kind, transpose)
    w = make(kind)
    d = op.disc_from(w)
    v = W.random_field(w.shape, 17)
    ref = op.apply_DT(d, v) if transpose else op.apply_D(d, v)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        x = dev(v)
        y = zeros(w.shape)
        ctx.apply_A(x, y, transpose)
        got = host(y)
    assert rel(got, ref) <= 1e-11, rel(got, ref)


@pytest.mark.parametrize("kind", ["small", "headline_24x16x8", "ragged_var_24x48x6", "radix3_192x96x12",
                                  "min_4x4x4", "radix5_var_50x80x100", "radix5_colcoef_100x50x8"])
def test_apply_S(kind):
    banner("apply_S", kind)
    w = make(kind).replace(rho=1.3, delta=0.6, obj_weights=1)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    v = W.random_field(w.shape, 5)
    ref = admm.apply_S(d, sc, v)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        y = zeros(w.shape)
        ctx.apply_S(dev(v), y)
        got = host(y)
    assert rel(got, ref) <= 1e-11, rel(got, ref)


@pytest.mark.parametrize("kind", OP_CASES)
@pytest.mark.parametrize("fp32", [0, 1])
def test_precond(kind, fp32):
    banner("precond", kind, fp32)
    w = make(kind).replace(rho=1.2, delta=0.5)
    d = op.disc_from(w)
    tab = pc.precond_tables(w, d)
    r = W.random_field(w.shape, 23)
    ref = pc.apply_precond(tab, r)
    prob, prm = fde.from_workload(w, precond_fp32=fp32)
    with fde.Context(prob, prm) as ctx:
        z = zeros(w.shape)
        ctx.precond(dev(r), z)
        got = host(z)
    tol = 2e-5 if fp32 else 1e-11
    assert rel(got, ref) <= tol, rel(got, ref)


@pytest.mark.parametrize("kind", ["small", "headline_24x16x8", "radix3_192x96x12", "min_4x4x4", "min_mixed_4x6x12",
                                  "radix5_var_50x80x100", "radix5_160x100x50"])
def test_krylov(kind):
    banner("krylov", kind)
    w = make(kind)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    tab = pc.precond_tables(w, d)
    b = W.random_field(w.shape, 8)
    x0 = 0.1 * W.random_field(w.shape, 9)
    xr, itr, relr, ok = admm.pcg(lambda v: admm.apply_S(d, sc, v), lambda v: pc.apply_precond(tab, v), b, x0,
                                 w.krylov_tol, w.krylov_maxit)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        x = dev(x0)
        it, relres, st = ctx.krylov(dev(b), x)
        got = host(x)
    assert st == fde.FDE_OK and ok
    assert abs(it - itr) <= 1, (it, itr)
    assert relres <= w.krylov_tol
    assert rel(got, xr) <= 1e-9, rel(got, xr)


def test_krylov_zero_rhs_returns_zero():
    banner("krylov zero rhs")
    w = make("small")
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        x = dev(W.random_field(w.shape, 1))
        it, relres, st = ctx.krylov(zeros(w.shape), x)
        assert it == 0 and st == fde.FDE_OK
        assert np.all(host(x) == 0.0)


def test_misaligned_fields_are_rejected_before_device_work():
    banner("misaligned fields")
    w = make("small")
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        buf = zeros((w.N + 1,))
        bad = buf[1:].view(w.shape)  # 8-byte offset
        y = zeros(w.shape)
        with pytest.raises(fde.FdeError) as e:
            ctx.apply_S(bad, y)
        assert e.value.status == fde.FDE_EINVAL and "16-byte aligned" in str(e.value)
        with pytest.raises(fde.FdeError) as e:
            state = {k: zeros(w.shape) for k in ("u", "zy", "zu", "p", "wy", "wu")}
            state["y"] = bad
            ctx.admm_solve(dev(w.yhat), state=state)
        assert e.value.status == fde.FDE_EINVAL
        # the context is still usable
        ctx.apply_S(dev(W.random_field(w.shape, 2)), y)
        assert np.isfinite(host(y)).all()


def test_time_pass_then_solve():
    """The pass timer covers all nine passes with their algorithmic byte
    counts, rejects a bad pass, and leaves the context usable."""
    banner("time_pass")
    w = make("ragged_var_24x48x6")
    prob, prm = fde.from_workload(w)
    n8 = 8.0 * w.N
    sb = (w.nx // 2 + 1) * w.ny * w.nt * 16.0
    expect = [2 * n8, 3 * n8, 2 * n8, 4 * n8, 6 * n8 + sb, 2 * sb, 2 * sb, 2 * sb, 2 * n8 + sb]
    with fde.Context(prob, prm) as ctx:
        for i in range(9):
            us, by = ctx.time_pass(i, 40)
            assert us > 0 and by == expect[i], (i, us, by)
        with pytest.raises(fde.FdeError) as e:
            ctx.time_pass(9, 5)
        assert e.value.status == fde.FDE_EINVAL
        d = op.disc_from(w)
        sc = admm.scalars(w, d)
        b = W.random_field(w.shape, 4)
        x = zeros(w.shape)
        it, relres, st = ctx.krylov(dev(b), x)
        assert st == fde.FDE_OK
        assert rel(admm.apply_S(d, sc, host(x)), b) <= 1e-9


@pytest.mark.parametrize("maxit", [2, 7, 13])
def test_krylov_maxit_reports_not_converged(maxit, monkeypatch):
    """The iteration limit stops PCG after exactly maxit iterations, whether a
    chunk is launched as graphs of four iterations, of one, or both (7, 13),
    and the iterate equals that of plain launches bitwise."""
    banner("krylov maxit", maxit)
    w = make("small").replace(krylov_maxit=maxit, krylov_tol=1e-30)
    b = W.random_field(w.shape, 2)
    out = []
    for mode in ("0", "1"):
        monkeypatch.setenv("FDE_NO_GRAPH", mode)
        prob, prm = fde.from_workload(w)
        with fde.Context(prob, prm) as ctx:
            x = zeros(w.shape)
            it, relres, st = ctx.krylov(dev(b), x)
            out.append(host(x))
        assert st == fde.FDE_ENOTCONV and it == maxit, (mode, st, it)
    assert np.array_equal(out[0], out[1])


def _admm_compare(w, fp32=0, tol=1e-7):
    prob, prm = fde.from_workload(w, precond_fp32=fp32)
    with fde.Context(prob, prm) as ctx:
        state, stats, status = ctx.admm_solve(dev(w.yhat), g=None if w.g is None else dev(w.g))
        got = {k: host(v) for k, v in state.items()}
    K = stats["admm_iters"]
    ref = admm.admm_solve(w)
    assert status == fde.FDE_OK and ref.converged
    assert abs(K - ref.iters) <= 1, (K, ref.iters)
    if K != ref.iters:
        ref = admm.admm_solve(w, iters=K)
    for k in ("y", "u", "zy", "zu", "p", "wy", "wu"):
        r = rel(got[k], getattr(ref, k))
        assert r <= tol, (k, r)
    # objective and dual infeasibility of the returned iterate (the oracle's
    # definitions evaluated on the GPU iterate)
    sc = admm.scalars(w, op.disc_from(w))
    J = kkt.objective(w, got["y"], got["u"])
    assert abs(stats["J"] - J) <= 1e-12 * max(1.0, abs(J)), (stats["J"], J)
    di = kkt.kkt_residuals(w, got["y"], got["u"], sc.psi * got["p"], sc.e_y * got["wy"],
                           sc.e_u * got["wu"])["dual_inf"]
    assert abs(stats["dual_inf"] - di) <= 1e-10 + 1e-8 * di, (stats["dual_inf"], di)
    return got, stats, ref


@pytest.mark.parametrize("kind", ["small", "small_mixed", "small_state"])
def test_admm_small(kind):
    banner("admm", kind)
    w = {"small": W.small, "small_mixed": W.small_mixed, "small_state": W.small_state}[kind]()
    got, stats, ref = _admm_compare(w)
    pol = kkt.polish(w, got["zy"], got["zu"])
    assert pol["ok"]


def edge_case(kind):
    if kind == "g_nonzero":
        return W.small_mixed(nx=12, ny=8, nt=6).replace(g=0.5 * W.random_field((6, 8, 12), 31))
    if kind == "free_control":
        return W.small_state(nx=12, ny=8, nt=6).replace(ua=-np.inf, ub=np.inf)
    if kind == "orders_near_1":
        return W.small_mixed(nx=12, ny=8, nt=6).replace(alpha=1.05, beta=1.1)
    raise KeyError(kind)


@pytest.mark.parametrize("kind", ["g_nonzero", "free_control", "orders_near_1"])
def test_admm_edge_cases(kind):
    """A nonzero FDE right-hand side g, an unbounded control (only the state
    bound active), and orders near 1 where the Riesz factor -1/(2 cos(a pi/2))
    is large."""
    banner("admm edge case", kind)
    w = edge_case(kind)
    got, stats, ref = _admm_compare(w)
    assert kkt.polish(w, got["zy"], got["zu"])["ok"]


def _admm_fixed(w, iters, tol=1e-7):
    prob, prm = fde.from_workload(w, admm_tol=0.0, admm_maxit=iters)
    with fde.Context(prob, prm) as ctx:
        state, stats, status = ctx.admm_solve(dev(w.yhat))
        got = {k: host(v) for k, v in state.items()}
    assert stats["admm_iters"] == iters
    ref = admm.admm_solve(w, iters=iters)
    for k in ("y", "u", "zy", "zu", "p", "wy", "wu"):
        r = rel(got[k], getattr(ref, k))
        assert r <= tol, (k, r)
    return got


def test_admm_psi_scaling_of_B_only():
    """psi_scaling = 2 (B = psi D, copies of u unscaled): 60 iterations."""
    banner("admm psi_scaling 2")
    _admm_fixed(W.small_mixed(nx=12, ny=8, nt=6).replace(psi_scaling=2), 60)


def test_operators_without_psi_scaling():
    banner("operators psi_scaling 0")
    w = var_fields(W.small(nx=24, ny=12, nt=6)).replace(psi_scaling=0)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    assert sc.psi == 1.0
    v = W.random_field(w.shape, 33)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        y = zeros(w.shape)
        ctx.apply_S(dev(v), y)
        assert rel(host(y), admm.apply_S(d, sc, v)) <= 1e-11
        ctx.precond(dev(v), y)
        assert rel(host(y), pc.apply_precond(pc.precond_tables(w, d), v)) <= 1e-11


def test_admm_paper_control_sign_exact_zero_optimum():
    """The headline shape with the paper's control sign (D y + u = g): D is an
    M-matrix, so u >= 0 forces y <= 0 <= yhat and the optimum is y = u = 0
    exactly.  200 iterations against the oracle, then a converged solve."""
    banner("admm ctrl_sign +1 zero optimum")
    w = W.headline(nx=12, ny=12, nt=6).replace(ctrl_sign=1.0)
    _admm_fixed(w, 200)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        state, stats, status = ctx.admm_solve(dev(w.yhat))
        y, u = host(state["y"]), host(state["u"])
    assert status == fde.FDE_OK
    assert np.abs(y).max() <= 1e-5 and np.abs(u).max() <= 1e-5, (np.abs(y).max(), np.abs(u).max())


@pytest.mark.parametrize("ycol", ["1", "0"])
def test_x_only_coefficients_both_y_pass_paths(monkeypatch, ycol):
    """Coefficient fields varying along x only (d+ and d- both): the
    per-column y-pass (two transforms per column pair, Hermitian separation)
    and the general variable-coefficient y-pass (FDE_YCOL=0) both match the
    oracle; ragged column tiles (nx = 24) and a radix-3 y length."""
    banner("x-only coefficients, FDE_YCOL", ycol)
    monkeypatch.setenv("FDE_YCOL", ycol)
    w = W.small(nx=24, ny=48, nt=6).replace(alpha=1.35, beta=1.65)
    w.dplus = W.coef_sine_x(24, 48)
    w.dminus = W.coef_sine_x(24, 48, amp=-0.3)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    v = W.random_field(w.shape, 51)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        y = zeros(w.shape)
        for tr, ref in ((False, op.apply_D(d, v)), (True, op.apply_DT(d, v))):
            ctx.apply_A(dev(v), y, tr)
            assert rel(host(y), ref) <= 1e-11, (tr, rel(host(y), ref))
        ctx.apply_S(dev(v), y)
        assert rel(host(y), admm.apply_S(d, sc, v)) <= 1e-11
    _admm_fixed(w.replace(ua=-5.0, ub=5.0), 40)


def test_admm_headline_shape_small():
    banner("admm headline 12x12x6")
    w = W.headline(nx=12, ny=12, nt=6)
    _admm_compare(w)


def test_admm_trapezoidal_rho():
    banner("admm trapezoidal")
    w = W.small_mixed(nx=12, ny=8, nt=6, obj_weights=1, rho=1.618, delta=0.4)
    _admm_compare(w)


def test_admm_resume_is_bitwise_continuation():
    """Running K iterations, then K more from the returned state, equals 2K at once."""
    banner("admm resume")
    w = W.small_mixed(nx=12, ny=8, nt=6).replace(admm_tol=0.0, admm_maxit=15)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        s1, _, _ = ctx.admm_solve(dev(w.yhat))
        s1, _, _ = ctx.admm_solve(dev(w.yhat), state=s1)
        a = {k: host(v) for k, v in s1.items()}
    prob2, prm2 = fde.from_workload(w.replace(admm_maxit=30))
    with fde.Context(prob2, prm2) as ctx:
        s2, st2, _ = ctx.admm_solve(dev(w.yhat))
        b = {k: host(v) for k, v in s2.items()}
    assert st2["admm_iters"] == 30
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_admm_deterministic():
    banner("admm determinism")
    w = W.small_mixed(nx=24, ny=16, nt=8).replace(admm_tol=0.0, admm_maxit=20)
    outs = []
    for _ in range(2):
        prob, prm = fde.from_workload(w)
        with fde.Context(prob, prm) as ctx:
            s, _, _ = ctx.admm_solve(dev(w.yhat))
            outs.append(host(s["y"]))
    assert np.array_equal(outs[0], outs[1])


def test_gradients_match_oracle_formula():
    banner("grad")
    w = W.small_mixed(nx=12, ny=8, nt=6).replace(alpha=1.4, beta=1.6)
    prob, prm = fde.from_workload(w)
    rng = np.random.Generator(np.random.PCG64(4))
    y = rng.standard_normal(w.shape)
    p = rng.standard_normal(w.shape)
    from oracle import grad

    psi = admm.scalars(w, op.disc_from(w)).psi
    gy, ga, gb = grad.gradients(w, y, psi * p)
    with fde.Context(prob, prm) as ctx:
        dy = zeros(w.shape)
        _, da, db = ctx.grad(dev(w.yhat), dev(y), dev(p), dyhat=dy)
        dyh = host(dy)
    assert rel(dyh, gy) <= 1e-14
    assert abs(da - ga) <= 1e-10 * abs(ga), (da, ga)
    assert abs(db - gb) <= 1e-10 * abs(gb), (db, gb)


def test_graph_replays_match_eager_launches(monkeypatch):
    """The PCG iteration replayed from a HIP graph gives bitwise the results
    of kernel-by-kernel launches, over several solves with eager work between."""
    banner("graph vs eager")
    w = make("headline_24x16x8")
    outs = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("FDE_NO_GRAPH", mode)
        prob, prm = fde.from_workload(w)
        with fde.Context(prob, prm) as ctx:
            res = []
            x = zeros(w.shape)
            for k in range(3):
                b = dev(W.random_field(w.shape, 30 + k))
                it, _, st = ctx.krylov(b, x)
                y = zeros(w.shape)
                ctx.apply_A(x, y)  # eager work between replays
                res.append((it, host(x), host(y)))
            outs[mode] = res
    for (i1, x1, y1), (i0, x0, y0) in zip(outs["1"], outs["0"]):
        assert i1 == i0
        assert np.array_equal(x1, x0) and np.array_equal(y1, y0)


@pytest.mark.parametrize("tiles", ["1,1,1", "2,2,2", "0,2,1"])
@pytest.mark.parametrize("kind", ["headline_24x16x8", "radix3_192x96x12", "long_1024x8x4", "tall_var_8x768x4",
                                  "tall_6x512x6", "deep_4x6x1024"])
def test_tile_variants_match_oracle(monkeypatch, tiles, kind):
    """Every column-tile variant the autotuner may pick gives the oracle's results."""
    banner("tiles", tiles, kind)
    monkeypatch.setenv("FDE_TILES", tiles)
    w = make(kind).replace(rho=1.3, delta=0.6)
    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    tab = pc.precond_tables(w, d)
    v = W.random_field(w.shape, 5)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        y = zeros(w.shape)
        ctx.apply_S(dev(v), y)
        z = zeros(w.shape)
        ctx.precond(dev(v), z)
        gs, gz = host(y), host(z)
    assert rel(gs, admm.apply_S(d, sc, v)) <= 1e-11
    assert rel(gz, pc.apply_precond(tab, v)) <= 1e-11


def test_autotune_then_solve_matches_oracle():
    banner("autotune")
    w = W.small_mixed(nx=24, ny=16, nt=8)
    prob, prm = fde.from_workload(w)
    with fde.Context(prob, prm) as ctx:
        ch = ctx.autotune()
        assert ch[0] >= 1 and 0 <= ch[1] <= 2 and 0 <= ch[2] <= 2
        assert ctx.autotune() == ch  # cached
        state, stats, status = ctx.admm_solve(dev(w.yhat))
        y = host(state["y"])
    ref = admm.admm_solve(w, iters=stats["admm_iters"])
    assert rel(y, ref.y) <= 1e-7


def test_convergence_test_placements_agree(monkeypatch):
    """The PCG convergence test fused into the preconditioner's y-forward pass
    and the stand-alone one-block test (used on large grids) stop PCG at the
    same iteration: Krylov solves and a short ADMM run are bitwise equal, and
    equal to the oracle."""
    banner("convergence test: fused vs separate")
    w = make("ragged_var_24x48x6").replace(ua=-5.0, ub=5.0, admm_tol=0.0, admm_maxit=8)
    b = W.random_field(w.shape, 44)
    out = []
    for sep in ("0", "1"):
        monkeypatch.setenv("FDE_CONV_SEPARATE", sep)
        prob, prm = fde.from_workload(w)
        with fde.Context(prob, prm) as ctx:
            x = zeros(w.shape)
            it, relres, st = ctx.krylov(dev(b), x)
            state, stats, _ = ctx.admm_solve(dev(w.yhat))
            out.append((it, host(x), {k: host(v) for k, v in state.items()}, stats["pcg_total"]))
    assert out[0][0] == out[1][0] and np.array_equal(out[0][1], out[1][1])
    assert out[0][3] == out[1][3]
    for k in out[0][2]:
        assert np.array_equal(out[0][2][k], out[1][2][k]), k
    ref = admm.admm_solve(w, iters=8)
    assert rel(out[1][2]["y"], ref.y) <= 1e-7
