"""Newton and backward-Euler drivers over vms_newton_step.

The loop control is host-side (the paper iterates Newton until the residual
is below a tolerance, Section 4.2, and marches the transient problem with
backward Euler, Section 4.1 Remark); every numerical step runs in the GPU
library.  States are device tensors updated in place:
  u [n_nodes, 4] float64 (vx, vy, vz, p), beta [n_elems, 3] float64.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import torch

from . import binding as B


@dataclass
class NewtonResult:
    converged: bool
    rnorms: list = field(default_factory=list)      # ||R_0||, ||R_1||, ...
    lin: list = field(default_factory=list)         # per-step solve info dicts
    seconds: float = 0.0


def set_dirichlet(u, dofs_dev, values_dev):
    """Write prescribed values into u (dofs are 4*node + c)."""
    u.view(-1).index_copy_(0, dofs_dev.long(), values_dev)


def forcing_term(k, rn, rn_prev, eta_prev, tol, r0, eta_max=0.1, gamma=0.9):
    """Linear tolerance of Newton step k (Eisenstat-Walker, second choice, with
    the usual safeguards).  Never asks for more than what brings ||R|| to tol ||R_0||."""
    if k == 0:
        eta = eta_max
    else:
        eta = gamma * (rn / rn_prev) ** 2
        if gamma * eta_prev ** 2 > 0.1:
            eta = max(eta, gamma * eta_prev ** 2)
        eta = min(eta, eta_max)
    return max(eta, 0.5 * tol * r0 / rn)


def newton_solve(ctx: B.Context, u, beta, Re, dt=0.0, u_prev=None, body=None, tol=1e-8, max_newton=25,
                 lin: B.SolveOpts | None = None, stream=None, raise_on_fail=True,
                 forcing: str = "fixed", method: str = "schur") -> NewtonResult:
    """Newton iterations until ||R_k|| <= tol ||R_0|| (FP64 residual).

    method="schur": Newton-Schur (condensed system, Section 5); method="full": Newton-Raphson
    on the uncondensed system (Section 4.2; the context needs full_system=True).
    forcing="fixed": every linear solve to lin.rtol.  forcing="ew": inexact
    Newton, linear tolerance from forcing_term() (never below lin.rtol)."""
    if method not in ("schur", "full"):
        raise ValueError(f"method must be 'schur' or 'full', not {method!r}")
    step = B.vms_newton_step if method == "schur" else B.vms_full_newton_step
    lin = lin if lin is not None else B.solve_opts()
    res = NewtonResult(converged=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r0 = None
    rn_prev = None
    eta = None
    rn = None
    for k in range(max_newton):
        if forcing == "ew" and rn is not None:
            eta = max(lin.rtol, forcing_term(k, rn, rn_prev, eta, tol, r0))
            lin.rtol, saved = eta, lin.rtol
        elif forcing == "ew":
            saved = lin.rtol
            eta = max(lin.rtol, 0.1)
            lin.rtol = eta
        else:
            saved = lin.rtol
        try:
            info = step(ctx, u, beta, Re, dt, u_prev, body, lin, stream)
        finally:
            lin.rtol = saved
        rn_prev = info.rnorm_before
        rn = info.rnorm_after
        if r0 is None:
            r0 = info.rnorm_before
            res.rnorms.append(r0)
        res.rnorms.append(info.rnorm_after)
        d = info.lin.as_dict()
        d["rtol"] = eta if eta is not None else lin.rtol
        res.lin.append(d)
        if info.rnorm_after <= tol * r0 or info.rnorm_after == 0.0:
            res.converged = True
            break
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    if not res.converged and raise_on_fail:
        raise B.VmsError(B.VMS_ENOCONV_NEWTON, f"Newton did not reach {tol:g}: {res.rnorms}")
    return res


def time_march(ctx: B.Context, u, beta, Re, dt, steps, bc_values_at, dofs_dev, tol=1e-8, lin=None, body=None,
               on_step=None, max_newton=25):
    """Backward Euler from the state in u.  bc_values_at(t) -> device float64
    values of the Dirichlet dofs at time t.  Returns the per-step results."""
    out = []
    u_prev = torch.empty_like(u)
    for n in range(steps):
        t_next = (n + 1) * dt
        u_prev.copy_(u)
        set_dirichlet(u, dofs_dev, bc_values_at(t_next))
        r = newton_solve(ctx, u, beta, Re, dt, u_prev, body, tol=tol, lin=lin, max_newton=max_newton)
        out.append(r)
        if on_step is not None:
            on_step(n, t_next, r)
    return out
