"""torch.autograd binding of the optimal value J*(yhat, alpha, beta).

Forward: one ADMM solve through the C ABI (fde_admm_solve); J is the
objective at the returned iterate.  Backward: fde_grad with the adjoint
transposed-Toeplitz solve, which gives dJ/dyhat = -J1 (y - yhat) and
dJ/dalpha, dJ/dbeta = lambda^T (dD/dalpha) y, ... (envelope theorem on the
Lagrangian of eq. (3.5)).  Both run in the library's kernels; this module
only passes arguments and applies the chain rule with the incoming scalar.
"""
from __future__ import annotations

import torch

from . import fde


class FDEObjective(torch.autograd.Function):
    """J* = FDEObjective.apply(yhat, alpha, beta, spec).

    yhat: float64 GPU tensor (nt, ny, nx); alpha, beta: 0-dim float64 tensors;
    spec: dict with the remaining problem fields (nx, ny, nt, gamma, bounds,
    tolerances ...) accepted by fde.make_problem / fde.make_params.
    """

    @staticmethod
    def forward(ctx, yhat, alpha, beta, spec):
        prob = fde.make_problem(spec["nx"], spec["ny"], spec["nt"], float(alpha), float(beta),
                                T=spec.get("T", 1.0), dplus=spec.get("dplus"), dminus=spec.get("dminus"),
                                ctrl_sign=spec.get("ctrl_sign", 1.0), psi_scaling=spec.get("psi_scaling", 1),
                                obj_weights=spec.get("obj_weights", 0))
        keys = ("delta", "rho", "ya", "yb", "ua", "ub", "krylov_tol", "krylov_maxit", "tol_mode", "admm_tol",
                "admm_maxit")
        prm = fde.make_params(spec["gamma"], **{k: spec[k] for k in keys if k in spec})
        c = fde.Context(prob, prm)
        state, stats, status = c.admm_solve(yhat.contiguous())
        ctx.fde = c
        ctx.stats = stats
        ctx.save_for_backward(yhat, state["y"], state["p"], state["wy"])
        return torch.tensor(stats["J"], dtype=torch.float64, device=yhat.device)

    @staticmethod
    def backward(ctx, g):
        yhat, y, p, wy = ctx.saved_tensors
        dyhat = torch.empty_like(yhat)
        _, da, db = ctx.fde.grad(yhat.contiguous(), y, p, wy, adjoint_solve=True, dyhat=dyhat)
        ctx.fde.close()
        ga = torch.tensor(da, dtype=torch.float64, device=yhat.device)
        gb = torch.tensor(db, dtype=torch.float64, device=yhat.device)
        return g * dyhat, g * ga, g * gb, None


def objective(yhat, alpha, beta, **spec):
    """Differentiable optimal value; see FDEObjective."""
    return FDEObjective.apply(yhat, alpha, beta, spec)


def spec_from_workload(w, **overrides):
    """The `spec` dict of a workload-like object (all fields but yhat, alpha, beta)."""
    spec = dict(nx=w.nx, ny=w.ny, nt=w.nt, T=w.T, dplus=w.dplus, dminus=w.dminus, ctrl_sign=w.ctrl_sign,
                psi_scaling=w.psi_scaling, obj_weights=w.obj_weights, gamma=w.gamma, delta=w.delta, rho=w.rho,
                ya=w.ya, yb=w.yb, ua=w.ua, ub=w.ub, krylov_tol=w.krylov_tol, krylov_maxit=w.krylov_maxit,
                admm_tol=w.admm_tol, admm_maxit=w.admm_maxit)
    spec.update(overrides)
    return spec
