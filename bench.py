"""Benchmark: ADMM hot path on the 256^2 x 64 headline grid, one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-full] [--no-cpu]

A step is one ADMM iteration of Algorithm 1 (right-hand side, the PCG solve
of the normal equations, recovery of p and u, box projection, dual updates
and residual maxima) over the synthetic headline workload: orders 1.3/1.7,
d+ = 1 + 0.5 sin(2 pi x), d- = 1, yhat = 16 e^t x(1-x) y(1-y), gamma 1e-6,
0 <= u <= 2, y <= 0.8, control as a source, delta = rho = 1, Krylov tol
1e-10, ADMM tol 1e-6, FP64.  W untimed iterations from a cold start are
followed by K timed ones; value = PCG iterations per second over the timed
region (inputs resident in HBM).  The cold-start ADMM solve (tolerance 1e-6,
iteration cap --full-cap) is timed as well, FP64 and with the FP32
preconditioner; at this grid and delta = rho = 1 the ADMM residual on the
control copy falls slowly, so the cap is normally reached and the record says
so ("converged": false, residuals).  Each PCG pass is timed with HIP events
for the roofline figure of the dominant kernel.  The batched legs run many
uneven instances for a fixed ADMM budget each (instances_per_s counts these
budgeted runs, not converged solves): in lockstep, stream-per-instance
concurrently, each in FP64 and with the FP32 preconditioner, and sequentially
in FP64.  The CPU oracle's PCG iteration on the same grid is timed on a
bounded sample.
Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TF = 78.6  # MI355X FP64 vector peak, TFLOP/s
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-full", action="store_true", help="skip the full cold-start solves")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=48)
    ap.add_argument("--full-cap", type=int, default=1500,
                    help="ADMM iteration cap of the cold-start solves (tolerance 1e-6)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-instances leg")
    ap.add_argument("--batch-cap", type=int, default=30, help="ADMM iterations per batched instance")
    ap.add_argument("--pass-reps", type=int, default=50, help="launches per pass for the per-pass timing")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's Table 5 protocol")
    ap.add_argument("--precision-iters", type=int, default=20,
                    help="ADMM iterations of the 1024^2 x 32 precision-form comparison")
    ap.add_argument("--variant-iters", type=int, default=100,
                    help="ADMM iterations of each preconditioner/ADMM variant on the headline grid")
    ap.add_argument("--diff-iters", type=int, default=30,
                    help="ADMM iterations of the 512^2 x 32 differentiation form before its backward pass")
    ap.add_argument("--admm-sweep", action="store_true",
                    help="only sweep the ADMM settings (psi scaling of the u copies, delta, rho) on the headline "
                         "grid: iterations and time to the 1e-4 and 1e-6 stopping tests; prints one JSON line")
    ap.add_argument("--sweep-cap", type=int, default=3000, help="ADMM iteration cap per setting of --admm-sweep")
    ap.add_argument("--lockstep-only", choices=["small", "mid"],
                    help="only the lockstep batch, FP64: the 256 small instances or the 64 mid-size ones, "
                         "--batch-cap ADMM iterations each; prints one JSON line (for kernel traces)")
    ap.add_argument("--passes-only", choices=["headline", "headline_fp32", "precision", "precision_fp32"],
                    help="only the in-solve per-pass timing on that grid (warmup W, then K timed ADMM "
                         "iterations); prints one JSON line (for kernel traces and counters)")
    return ap.parse_args()


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(w, iters):
    """The oracle's PCG (dense Toeplitz / dense DFT, FP64 NumPy) on the same grid:
    `iters` iterations from a seeded right-hand side."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import workloads as W
    from oracle import admm, precond
    from oracle import operator as op

    d = op.disc_from(w)
    sc = admm.scalars(w, d)
    tab = precond.precond_tables(w, d)
    b = W.random_field(w.shape, 99)
    t0 = time.perf_counter()
    admm.pcg(lambda v: admm.apply_S(d, sc, v), lambda v: precond.apply_precond(tab, v), b, np.zeros(w.shape),
             0.0, iters)
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"value": iters / dt, "unit": "PCG iters/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{iters} PCG iterations of the oracle on the 256x256x64 headline grid "
                      f"(S apply + no-FFT preconditioner), {dt:.1f} s"}


COPY_BYTES = 256 << 20  # plain device copy: achievable-bandwidth and counter calibration


def copy_calibration(torch, reps=5):
    """A plain device-to-device copy of COPY_BYTES (torch's copy kernel): the
    achievable read+write bandwidth, and the known-size kernel against which the
    FETCH_SIZE / WRITE_SIZE counters of the roofline traffic are scaled."""
    n = COPY_BYTES // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    return {"bytes_per_copy": 2 * COPY_BYTES, "us": round(us, 2), "GB/s": round(2 * COPY_BYTES / us / 1e3, 1)}


COMMON_SOURCES = ["paper_1907_13428_amd/csrc/fde_fft.hpp", "paper_1907_13428_amd/csrc/fde_internal.hpp",
                  "paper_1907_13428_amd/csrc/fde_reduce.hpp"]


def kernel_sources(pass_name):
    """The source files that define the kernel of a PCG pass."""
    own = "k_toeplitz.hip" if pass_name.split("_")[0] in ("xpass", "ypass") else "k_precond.hip"
    return ["paper_1907_13428_amd/csrc/" + own] + COMMON_SOURCES


def kernel_source_hash(pass_name):
    import hashlib

    h = hashlib.sha256()
    for f in kernel_sources(pass_name):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(pass_name, tile_width=None):
    """Memory-side bytes per launch of the dominant kernel from the committed
    counter summary profiles/traffic_<pass>_headline_256x256x64.json
    (FETCH_SIZE and WRITE_SIZE runs scaled by the copy kernel; they count the
    L2's traffic to the memory side, last-level cache hits included), or None
    when there is none for this pass or the kernel sources have changed since
    the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{pass_name}_headline_256x256x64.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("pass") != pass_name or rec.get("source_sha256") != kernel_source_hash(pass_name):
        return None
    return rec.get("traffic_bytes")


def in_solve_passes(ctx, yhat, state, torch):
    """Per-pass figures of the PCG iteration measured inside ADMM iterations
    that continue from `state` (the context's admm_maxit of them): mean kernel
    duration per launch from events bound to each dispatch, algorithmic bytes
    per launch, GB/s, and the pass's share of the PCG passes' GPU time."""
    ctx.pass_timing(True)
    ctx.admm_solve(yhat, state=state)
    torch.cuda.synchronize()
    stats = ctx.pass_stats()
    ctx.pass_timing(False)
    total = sum(us * n for us, n, _ in stats.values())
    out = {}
    for name, (us, n, by) in stats.items():
        out[name] = {"us": round(us, 2), "launches": n, "bytes": by, "GB/s": round(by / us / 1e3, 1),
                     "share": round(us * n / total, 4)}
    return out


def passes_only_leg(fde, torch, grid, warmup, steps):
    """The in-solve per-pass table alone: `warmup` ADMM iterations from zero,
    then `steps` more with pass timing, on the headline grid or the 1024^2 x 32
    precision form, each in FP64 or with the FP32 preconditioner."""
    import workloads as W

    w = W.headline() if grid.startswith("headline") else W.precision()
    fp32 = 1 if grid.endswith("_fp32") else 0
    yhat = torch.from_numpy(w.yhat).to("cuda")
    prob, prm = fde.from_workload(w, precond_fp32=fp32, admm_tol=0.0, admm_maxit=max(warmup, 1))
    with fde.Context(prob, prm) as ctx:
        tiles = ctx.autotune()
        state, _, _ = ctx.admm_solve(yhat)
        ctx.set_params(fde.from_workload(w, precond_fp32=fp32, admm_tol=0.0, admm_maxit=steps)[1])
        passes = in_solve_passes(ctx, yhat, state, torch)
    return {"grid": grid, "shape": [w.nx, w.ny, w.nt], "autotune": tiles, "warmup": warmup, "steps": steps,
            "passes": passes, "copy_kernel": copy_calibration(torch)}


def paper_table5_leg(fde, torch):
    """The paper's test problem and protocol (Sec. 6.1; Caputo order 0.7,
    Riesz orders 1.3, box on both variables, dynamic Krylov tolerance, PCG from
    zero, ADMM tolerance 1e-4) at the Table 5 grid sizes, FP64 on the GPU,
    beside the printed figures (MATLAB on a CPU).  Each size also runs the
    generalized ADMM of Sec. 3.3.2 (step 1, R_y = I - J1, R_u = gamma I - J2),
    Algorithm 1 with the matching preconditioner of eq. (3.11), and Algorithm 1
    with the MINRES x-step (merged system, K~ of eq. (3.12))."""
    import workloads as W

    with open(os.path.join(ROOT, "tests", "golden", "paper_table5.json")) as f:
        rec = json.load(f)

    def run(w, n):
        prob, prm = fde.from_workload(w)
        yhat = torch.from_numpy(w.yhat).to("cuda")
        with fde.Context(prob, prm) as ctx:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            state, st, status = ctx.admm_solve(yhat)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            # discrete L2 misfit: trapezoidal in time (1/2 on the last level), sum in space
            h = 1.0 / (n + 1)
            e2 = ((state["y"] - yhat) ** 2).sum(dim=(1, 2))
            e2[-1] *= 0.5
            el2 = float(torch.sqrt(h * h * (w.T / w.nt) * e2.sum()))
        return {"converged": status == 0, "admm_iters": st["admm_iters"],
                "pcg_avg": round(st["pcg_total"] / max(st["admm_iters"], 1), 2), "E_L2": round(el2, 4),
                "dual_inf": st["dual_inf"], "s": round(dt, 4)}

    rows = []
    for row in (dict(zip(rec["columns"], r)) for r in rec["rows"]):
        w = W.paper_test(row["n"], delta=row["delta"])
        r = run(w, row["n"])
        rows.append({"n": row["n"], "delta": row["delta"], "converged": r["converged"],
                     "admm_iters": r["admm_iters"], "paper_admm_iters": row["admm_iters"],
                     "pcg_avg": r["pcg_avg"], "paper_pcg_avg": row["pcg_avg"], "E_L2": r["E_L2"],
                     "paper_E_L2": row["E_L2"], "dual_inf": r["dual_inf"], "paper_dual_inf": row["dual_inf"],
                     "s": r["s"], "paper_s": row["time_s"],
                     "generalized_admm": run(w.replace(prox=1, rho=1.0), row["n"]),
                     "matching_precond": run(w.replace(precond_kind=1), row["n"]),
                     "minres_xstep": run(w.replace(krylov_solver=1), row["n"])})
    return {"rows": rows, "paper_times": rec["time_note"]}


SWEEP_DELTAS = (0.01, 0.03, 0.1, 0.4, 2.0, 10.0, 100.0)


SWEEP_TOLS = (1e-2, 1e-3, 1e-4, 1e-6)


def admm_sweep_leg(fde, torch, w, yhat, cap):
    """ADMM settings on the headline grid (Alg. 1, Sec. 6.1): the psi scaling
    of the u copies (1: e_u = psi as in Sec. 6.1; 2: the constraint scaled,
    the copies not), delta from the paper's pool of Sec. 6 and below it, and
    rho in {1, 1.618}.  Each setting runs from zero to the stopping test at
    1e-2, then resumes from that state to 1e-3, 1e-4 and 1e-6 in turn
    (resuming is exact), with at most `cap` iterations in all.  FP64."""
    rows = []
    for ps in (1, 2):
        for rho in (1.0, 1.618):
            for delta in SWEEP_DELTAS:
                wl = w.replace(psi_scaling=ps, delta=delta, rho=rho)
                rec = {"psi_scaling": ps, "rho": rho, "delta": delta}
                it = pcg = 0
                t = 0.0
                state = None
                res = None
                prob, prm = fde.from_workload(wl, admm_tol=SWEEP_TOLS[0], admm_maxit=cap)
                with fde.Context(prob, prm) as c:
                    for tol in SWEEP_TOLS:
                        key = "%.0e" % tol
                        if it >= cap:
                            rec["it_" + key] = rec["s_" + key] = None
                            continue
                        c.set_params(fde.from_workload(wl, admm_tol=tol, admm_maxit=cap - it)[1])
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        state, st, status = c.admm_solve(yhat, state=state)
                        torch.cuda.synchronize()
                        t += time.perf_counter() - t0
                        it += st["admm_iters"]
                        pcg += st["pcg_total"]
                        res = [st["r_p"], st["r_y"], st["r_u"]]
                        ok = status == 0
                        rec["it_" + key] = it if ok else None
                        rec["s_" + key] = round(t, 3) if ok else None
                        if not ok:
                            it = cap
                rec.update({"iters": it, "pcg_total": pcg, "s": round(t, 3),
                            "residuals": [float("%.3e" % r) for r in res]})
                progress(f"sweep {rec}")
                rows.append(rec)
    return {"grid": [w.nx, w.ny, w.nt], "cap": cap, "rows": rows}


def differentiation_leg(fde, torch, iters):
    """The 512^2 x 32 differentiation form (orders 1.4/1.6, sinusoid-sum
    target, gamma 1e-4, |u| <= 1): `iters` ADMM iterations from zero (the
    forward pass), then the backward pass: gradients of the optimal value with
    the adjoint solve D^T lambda = -J1 (y - yhat) - w_y (backward time stepping,
    BiCGSTAB per step) and, for comparison, with lambda = psi p from the ADMM
    multiplier (envelope form, no solve)."""
    import workloads as W

    w = W.differentiation()
    yhat = torch.from_numpy(w.yhat).to("cuda")
    prob, prm = fde.from_workload(w, admm_tol=0.0, admm_maxit=iters)
    rec = {"grid": [w.nx, w.ny, w.nt], "admm_iters": iters}
    with fde.Context(prob, prm) as ctx:
        ctx.autotune()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        state, st, _ = ctx.admm_solve(yhat)
        torch.cuda.synchronize()
        rec["forward_s"] = round(time.perf_counter() - t0, 3)
        dy = torch.empty_like(yhat)
        lam = torch.empty_like(yhat)
        for tag, adj in (("backward_adjoint_solve", True), ("backward_envelope", False)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, da, db = ctx.grad(yhat, state["y"], state["p"], state["wy"], adjoint_solve=adj, dyhat=dy, lam=lam)
            torch.cuda.synchronize()
            rec[tag] = {"s": round(time.perf_counter() - t0, 4), "dJ_dalpha": da, "dJ_dbeta": db}
    return rec


def paper_tables_leg(fde, torch):
    """Tables 2, 3, 4, 6 and 7 of the paper (Sec. 6.2; all on the 50^3 grid):
    the rows of tests/golden/paper_tables.json under the Sec. 6.1 protocol, FP64
    on the GPU, beside the printed figures (MATLAB on a CPU)."""
    import workloads as W

    with open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")) as f:
        rec = json.load(f)
    bound = lambda v: -math.inf if v == "-inf" else float(v)
    rows = []
    for row in (dict(zip(rec["columns"], r)) for r in rec["rows"]):
        n = row["n"]
        w = W.paper_test(n, alpha_t=row["alpha"], beta=row["beta"], gamma=row["gamma"], ya=bound(row["ya"]),
                         ua=bound(row["ua"]), delta=row["delta"])
        prob, prm = fde.from_workload(w)
        yhat = torch.from_numpy(w.yhat).to("cuda")
        with fde.Context(prob, prm) as ctx:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            state, st, status = ctx.admm_solve(yhat)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            h = 1.0 / (n + 1)
            e2 = ((state["y"] - yhat) ** 2).sum(dim=(1, 2))
            e2[-1] *= 0.5
            el2 = float(torch.sqrt(h * h * (w.T / w.nt) * e2.sum()))
        rows.append({"table": row["table"], "alpha": row["alpha"], "beta": row["beta"], "gamma": row["gamma"],
                     "ya": row["ya"], "ua": row["ua"], "delta": row["delta"], "converged": status == 0,
                     "admm_iters": st["admm_iters"], "paper_admm_iters": row["admm_iters"],
                     "pcg_avg": round(st["pcg_total"] / max(st["admm_iters"], 1), 2),
                     "paper_pcg_avg": row["pcg_avg"], "E_L2": round(el2, 4), "paper_E_L2": row["E_L2"],
                     "dual_inf": st["dual_inf"], "paper_dual_inf": row["dual_inf"], "s": round(dt, 4),
                     "paper_s": row["time_s"]})
    return {"rows": rows, "paper_times": rec["time_note"]}


def contrast_leg(fde, torch, iters):
    """The headline grid with d+ = 1 + c sin(2 pi x), c in {0.5, 0.9, 0.99}:
    Krylov iterations per x-step and time of `iters` ADMM iterations with S~
    (precond_kind 0) and with the diagonally scaled S~ (precond_kind 2)."""
    import workloads as W

    rec = {"admm_iters": iters}
    for amp in (0.5, 0.9, 0.99):
        w = W.headline()
        w.dplus = W.coef_sine_x(w.nx, w.ny, amp=amp)
        yh = torch.from_numpy(w.yhat).to("cuda")
        row = {}
        for tag, kind in (("S~", 0), ("S~diag", 2)):
            prob, prm = fde.from_workload(w.replace(precond_kind=kind), admm_tol=0.0, admm_maxit=iters)
            with fde.Context(prob, prm) as c:
                c.autotune()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st, _ = c.admm_solve(yh)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
            row[tag] = {"pcg_avg": round(st["pcg_total"] / st["admm_iters"], 2), "s": round(t, 3),
                        "pcg_iters_per_s": round(st["pcg_total"] / t, 1)}
        row["krylov_ratio"] = round(row["S~diag"]["pcg_avg"] / row["S~"]["pcg_avg"], 3)
        row["time_ratio"] = round(row["S~diag"]["s"] / row["S~"]["s"], 3)
        rec[f"c={amp}"] = row
    return rec


def batch_modes(fde, torch, ws, cap, modes):
    """Time fde_batch_solve over the instances ws (each run for `cap` ADMM
    iterations) in each (tag, fp32, mode) of `modes`."""
    yh = [torch.from_numpy(w.yhat).to("cuda") for w in ws]
    rec = {"instances": len(ws), "points": sum(w.N for w in ws), "admm_iters_per_instance": cap}
    for tag, fp32, mode in modes:
        probs, prms = zip(*[fde.from_workload(w, precond_fp32=fp32, admm_maxit=cap) for w in ws])
        with fde.Batch(list(probs), list(prms)) as b:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, stats, _ = b.solve(yh, concurrent=(mode != "sequential"), lockstep=(mode == "lockstep"))
            dt = time.perf_counter() - t0
        pcg = sum(s["pcg_total"] for s in stats)
        rec[tag] = {"s": round(dt, 3), "instances_per_s": round(len(ws) / dt, 2), "pcg_iters_per_s": round(pcg / dt, 1),
                    "pcg_total": pcg}
    return rec


def batched_leg(fde, torch, cap):
    """64 uneven instances (sizes 64..512, nt 16/32, random orders and gamma, GRF
    targets), each run for `cap` ADMM iterations: in lockstep (the Krylov
    iterations of all instances as batched pass launches), in the
    stream-per-instance concurrent mode, both FP64 and with the FP32
    preconditioner, and sequentially in FP64."""
    import workloads as W

    rec = batch_modes(fde, torch, W.batched(), cap,
                      (("lockstep_fp32_precond", 1, "lockstep"), ("lockstep_fp64", 0, "lockstep"),
                       ("concurrent_fp32_precond", 1, "concurrent"), ("concurrent_fp64", 0, "concurrent"),
                       ("sequential_fp64", 0, "sequential")))
    # the batched form alone (FP64 both ways), and with the FP32 preconditioner; the
    # stream-per-instance concurrent mode beside it
    rec["speedup_lockstep_fp64"] = round(rec["sequential_fp64"]["s"] / rec["lockstep_fp64"]["s"], 3)
    rec["speedup_concurrency_fp64"] = round(rec["sequential_fp64"]["s"] / rec["concurrent_fp64"]["s"], 3)
    rec["speedup"] = round(rec["sequential_fp64"]["s"] / rec["lockstep_fp32_precond"]["s"], 3)
    return rec


def batched_small_leg(fde, torch, cap):
    """256 small uneven instances (16..64 nodes per axis, nt 8/16; 4.4 M points in
    all), each run for `cap` ADMM iterations, FP64: lockstep, concurrent and
    sequential."""
    import workloads as W

    rec = batch_modes(fde, torch, W.batched_small(), cap,
                      (("lockstep_fp64", 0, "lockstep"), ("concurrent_fp64", 0, "concurrent"),
                       ("sequential_fp64", 0, "sequential")))
    rec["speedup_lockstep_fp64"] = round(rec["sequential_fp64"]["s"] / rec["lockstep_fp64"]["s"], 3)
    rec["speedup_concurrency_fp64"] = round(rec["sequential_fp64"]["s"] / rec["concurrent_fp64"]["s"], 3)
    return rec


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU; runs on several GPUs are not supported",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    import workloads as W
    from paper_1907_13428_amd import fde

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    w = W.headline()
    yhat = torch.from_numpy(w.yhat).to("cuda")
    if a.admm_sweep:
        print(json.dumps({"admm_sweep": admm_sweep_leg(fde, torch, w, yhat, a.sweep_cap)}), flush=True)
        return
    if a.passes_only:
        print(json.dumps(passes_only_leg(fde, torch, a.passes_only, a.warmup, a.steps)), flush=True)
        return
    if a.lockstep_only:
        import workloads as W

        ws = W.batched_small() if a.lockstep_only == "small" else W.batched()
        rec = batch_modes(fde, torch, ws, a.batch_cap, (("lockstep_fp64", 0, "lockstep"),))
        print(json.dumps({"lockstep": a.lockstep_only, **rec}), flush=True)
        return
    out = {"metric": "PCG iters/s + ADMM solve time, 256^2x64 grid; HBM GB/s; FP32-precond vs FP64",
           "unit": "PCG iters/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic"}

    # ---- timed ADMM iterations (FP64) -------------------------------------
    prob, prm = fde.from_workload(w, admm_tol=0.0, admm_maxit=max(a.warmup, 1))
    ctx = fde.Context(prob, prm)
    out["autotune"] = ctx.autotune()
    progress(f"warmup {a.warmup} ADMM iterations")
    state, st_w, _ = ctx.admm_solve(yhat)
    ctx.set_params(fde.from_workload(w, admm_tol=0.0, admm_maxit=a.steps)[1])
    torch.cuda.synchronize()
    progress(f"timing {a.steps} ADMM iterations")
    t0 = time.perf_counter()
    state, st, _ = ctx.admm_solve(yhat, state=state)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["value"] = st["pcg_total"] / dt
    out["value_window"] = f"ADMM iterations {a.warmup + 1}..{a.warmup + a.steps} of a cold start"
    out["ms_per_step"] = 1e3 * dt / a.steps
    out["pcg_per_admm_iter"] = st["pcg_total"] / a.steps
    out["phase_s_per_step"] = {"rhs": round(st["t_rhs"] / a.steps, 6), "krylov": round(st["t_krylov"] / a.steps, 6),
                               "update": round(st["t_update"] / a.steps, 6)}

    # ---- per-pass kernel durations inside the solve ------------------------
    # The same K ADMM iterations again from the reached state, the PCG passes as
    # plain launches with HIP events bound to each pass's own dispatch.
    progress(f"pass timing over {a.steps} ADMM iterations")
    passes = in_solve_passes(ctx, yhat, state, torch)
    # The dominant pass has the largest share of the passes' GPU time.  Passes
    # within 2% of that share are a tie (at the headline the y-pass of B^T and
    # the preconditioner's x-forward pass): the roofline then names the one
    # furthest from its peak and lists the others beside it.
    top = max(p["share"] for p in passes.values())
    tied = [k for k in passes if passes[k]["share"] >= 0.98 * top]
    dom = min(tied, key=lambda k: passes[k]["GB/s"])
    copy = copy_calibration(torch)
    achieved = passes[dom]["GB/s"]
    out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": measured_traffic(dom, out["autotune"][0]),
                       "bytes_per_launch": passes[dom]["bytes"], "us_per_launch": passes[dom]["us"],
                       "launches": passes[dom]["launches"], "copy_kernel": copy,
                       "tied_with": {k: {"share": passes[k]["share"], "GB/s": passes[k]["GB/s"],
                                         "frac": round(passes[k]["GB/s"] / HBM_PEAK_GBS, 4)}
                                     for k in tied if k != dom}}
    out["pcg_iteration_passes"] = passes
    # The line passes are FP64-VALU-heavy FFTs: nominal FFT flops (5 L log2 L
    # per complex transform of length L = 2n) per launch against the FP64
    # vector peak.  Headline: x-lines carry d+(x) (three transforms per pair of
    # lines); y-lines are constant-coefficient per column (two per pair).
    def fft_flops(n_lines, L, per_pair):
        return (n_lines / 2) * per_pair * 5.0 * L * math.log2(L)

    alu = {}
    for name, lines, L, tr in (("xpass_B", w.ny * w.nt, 2 * w.nx, 3), ("xpass_BT", w.ny * w.nt, 2 * w.nx, 3),
                               ("ypass_B", w.nx * w.nt, 2 * w.ny, 2), ("ypass_BT", w.nx * w.nt, 2 * w.ny, 2)):
        fl = fft_flops(lines, L, tr)
        tf = fl / passes[name]["us"] / 1e6
        alu[name] = {"nominal_fft_flops": fl, "TFLOP/s": round(tf, 1), "frac_fp64_peak": round(tf / FP64_PEAK_TF, 3)}
    out["line_passes_alu"] = {"peak_TFLOP/s": FP64_PEAK_TF, "passes": alu}
    pcg_pass_us = sum(p["us"] for p in passes.values())
    pcg_bytes = sum(p["bytes"] for p in passes.values())
    out["pcg_iteration_model"] = {"us": round(pcg_pass_us, 1), "GB": round(pcg_bytes / 1e9, 4),
                                  "GB/s": round(pcg_bytes / pcg_pass_us / 1e3, 1)}
    ctx.close()

    # ---- full cold-start solves: FP64 and FP32 preconditioner ---------------
    if not a.no_full:
        for tag, fp32 in (("fp64", 0), ("fp32_precond", 1)):
            progress(f"full ADMM solve ({tag})")
            prob, prm = fde.from_workload(w, precond_fp32=fp32, admm_maxit=a.full_cap)
            with fde.Context(prob, prm) as c2:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s2, st2, status = c2.admm_solve(yhat)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                if fp32 == 0:
                    y64 = s2["y"].clone()
                    u64 = s2["u"].clone()
                rec = {"admm_solve_s": round(t, 3), "admm_iters": st2["admm_iters"], "admm_cap": a.full_cap,
                       "pcg_total": st2["pcg_total"], "pcg_iters_per_s": round(st2["pcg_total"] / t, 1),
                       "ms_per_admm_iter": round(1e3 * t / st2["admm_iters"], 3), "converged": status == 0,
                       "residuals": [st2["r_p"], st2["r_y"], st2["r_u"]], "dual_inf": st2["dual_inf"],
                       "J": st2["J"], "phase_s": {"rhs": round(st2["t_rhs"], 4), "krylov": round(st2["t_krylov"], 4),
                                                  "update": round(st2["t_update"], 4)}}
                if fp32:
                    rec["rel_diff_y_vs_fp64"] = float(torch.linalg.norm(s2["y"] - y64) / torch.linalg.norm(y64))
                    rec["rel_diff_u_vs_fp64"] = float(torch.linalg.norm(s2["u"] - u64) / torch.linalg.norm(u64))
                out[tag] = rec
        out["admm_solve_s"] = out["fp64"]["admm_solve_s"]
        out["pcg_iters_per_s_whole_solve"] = out["fp64"]["pcg_iters_per_s"]

        # Krylov counts on the variable-coefficient headline grid: S~ (eq. (3.10))
        # against the matching S^ (eq. (3.11)), under Algorithms 1 and 2, and the
        # MINRES x-step on the merged system with K~ (eq. (3.12))
        progress("preconditioner and ADMM variants")
        var = {}
        # (the headline's J1 = I, so Algorithm 2 takes c_y = 1.5, c_u = 10 gamma: R_y, R_u nonzero)
        alg2 = dict(prox=1, prox_cy=1.5, prox_cu=10 * w.gamma)
        for tag, kw in (("S~_alg1", {}), ("S^_alg1", dict(precond_kind=1)), ("S~diag_alg1", dict(precond_kind=2)),
                        ("S~_alg2", alg2),
                        ("S^_alg2", dict(alg2, precond_kind=1)), ("minres_K~_alg1", dict(krylov_solver=1))):
            prob, prm = fde.from_workload(w.replace(**kw), admm_tol=0.0, admm_maxit=a.variant_iters)
            with fde.Context(prob, prm) as c3:
                c3.autotune()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st3, _ = c3.admm_solve(yhat)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
            var[tag] = {"admm_iters": st3["admm_iters"], "pcg_avg": round(st3["pcg_total"] / st3["admm_iters"], 2),
                        "s": round(t, 3), "residuals": [st3["r_p"], st3["r_y"], st3["r_u"]]}
        out["variants_headline"] = var
        progress("coefficient contrast: S~ against the diagonally scaled S~")
        out["contrast_headline"] = contrast_leg(fde, torch, a.variant_iters)

    # ---- precision form: 1024^2 x 32, FP32 preconditioner against FP64 ----------
    if not a.no_full:
        progress("precision form 1024^2 x 32: FP64 and FP32 preconditioner")
        wp = W.precision()
        yp = torch.from_numpy(wp.yhat).to("cuda")
        rec = {"grid": [wp.nx, wp.ny, wp.nt], "admm_iters": a.precision_iters}
        sol = {}
        for tag, fp32 in (("fp64", 0), ("fp32_precond", 1)):
            prob, prm = fde.from_workload(wp, precond_fp32=fp32, admm_tol=0.0, admm_maxit=a.precision_iters)
            with fde.Context(prob, prm) as c4:
                c4.autotune()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s4, st4, _ = c4.admm_solve(yp)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                sol[tag] = (s4["y"].clone(), s4["u"].clone())
            rec[tag] = {"s": round(t, 3), "pcg_total": st4["pcg_total"],
                        "pcg_iters_per_s": round(st4["pcg_total"] / t, 1)}
        for tag in ("precision", "precision_fp32"):
            progress(f"pass timing, {tag}")
            rec["passes_" + tag] = passes_only_leg(fde, torch, tag, 2, 3)["passes"]
        (y64, u64), (y32, u32) = sol["fp64"], sol["fp32_precond"]
        rec["rel_diff_y"] = float(torch.linalg.norm(y32 - y64) / torch.linalg.norm(y64))
        rec["rel_diff_u"] = float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64))
        out["precision_form"] = rec
        del sol, y64, u64, y32, u32, yp

    # ---- the paper's own test problem and protocol (Table 5 sizes) -----------
    if not a.no_paper:
        progress("paper test problem, Table 5 sizes")
        out["paper_table5"] = paper_table5_leg(fde, torch)
        progress("paper test problem, Tables 2, 3, 4, 6, 7")
        out["paper_tables"] = paper_tables_leg(fde, torch)

    # ---- differentiation form: forward ADMM and the backward pass --------------
    if not a.no_full:
        progress("differentiation form 512^2 x 32: forward and backward")
        out["differentiation"] = differentiation_leg(fde, torch, a.diff_iters)

    # ---- batched form: 64 uneven instances, concurrent vs sequential ---------
    if not a.no_batch:
        progress("batched instances")
        out["batched"] = batched_leg(fde, torch, a.batch_cap)
        progress("batched small instances")
        out["batched_small"] = batched_small_leg(fde, torch, a.batch_cap)

    out["config"] = {"workload": "headline_256x256x64", "nx": 256, "ny": 256, "nt": 64, "alpha": 1.3, "beta": 1.7,
                     "gamma": 1e-6, "delta": 1.0, "rho": 1.0, "krylov_tol": 1e-10, "admm_tol": 1e-6,
                     "precond": "fp64"}
    if not a.no_cpu:
        progress("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
