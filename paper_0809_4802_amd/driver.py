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


def newton_solve(ctx: B.Context, u, beta, Re, dt=0.0, u_prev=None, body=None, tol=1e-8, max_newton=25,
                 lin: B.SolveOpts | None = None, stream=None, raise_on_fail=True) -> NewtonResult:
    """Newton-Schur iterations until ||R_k|| <= tol ||R_0|| (FP64 residual)."""
    lin = lin if lin is not None else B.solve_opts()
    res = NewtonResult(converged=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r0 = None
    for _ in range(max_newton):
        info = B.vms_newton_step(ctx, u, beta, Re, dt, u_prev, body, lin, stream)
        if r0 is None:
            r0 = info.rnorm_before
            res.rnorms.append(r0)
        res.rnorms.append(info.rnorm_after)
        res.lin.append(info.lin.as_dict())
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
