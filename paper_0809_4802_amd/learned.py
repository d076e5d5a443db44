"""Training loop of the learned block-Jacobi correction (host orchestration).

Samples are residuals the method's own GMRES solves produce (the restart
residuals logged by vms_gmres_solve); every forward, backward and Adam step
runs in the library's kernels (vms_pc_train_step).
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


def init_weights(seed=1, device="cuda:0"):
    """Glorot-uniform first layer, zero output layer: the network starts as plain block-Jacobi."""
    rng = np.random.default_rng(seed)
    lim = np.sqrt(6.0 / (B.PC_NIN + B.PC_NHID))
    w = np.zeros(B.PC_NWEIGHTS, dtype=np.float32)
    w[:B.PC_NHID * B.PC_NIN] = rng.uniform(-lim, lim, size=B.PC_NHID * B.PC_NIN)
    return torch.from_numpy(w).to(device)


def collect_samples(ctx: B.Context, A, b, n_samples=8, cycle_iters=30, restart=None):
    """Restart residuals of a short GMRES(restart) run on A x = b (block-Jacobi)."""
    restart = restart or cycle_iters
    log = torch.zeros((n_samples, ctx.n_nodes, 4), dtype=torch.float32, device=ctx.device)
    x = ctx.new_vec()
    _, info = B.vms_gmres_solve(ctx, A, b, x, B.solve_opts(restart=restart, rtol=1e-14,
                                                            max_iters=cycle_iters * (n_samples - 1),
                                                            log_residuals=log), allow_noconv=True)
    return log[:max(1, info.logged)].contiguous()


def train(ctx: B.Context, data, steps=200, lr=1e-3, batch=8, seed=1, weights=None, log_every=0):
    """data: list of (bsr_vals, samples[k, n_nodes, 4]).  Returns (weights, loss history)."""
    rng = np.random.default_rng(seed)
    w = init_weights(seed, ctx.device) if weights is None else weights
    state = torch.zeros(2 * B.PC_NWEIGHTS, dtype=torch.float32, device=ctx.device)
    loss = torch.zeros(1, dtype=torch.float32, device=ctx.device)
    hist = []
    for step in range(1, steps + 1):
        A, S = data[rng.integers(len(data))]
        k = min(batch, S.shape[0])
        idx = torch.from_numpy(rng.choice(S.shape[0], size=k, replace=False)).to(ctx.device)
        rb = S.index_select(0, idx).contiguous()
        B.vms_pc_train_step(ctx, A, rb, w, state, step, lr, None, loss)
        hist.append(float(loss.item()))
        if log_every and step % log_every == 0:
            print(f"train step {step}: loss {hist[-1]:.4f}", flush=True)
    return w, hist


def collect_newton_data(ctx: B.Context, u, beta, Re, dt=0.0, u_prev=None, body=None, tol=1e-8, max_newton=20,
                        lin: B.SolveOpts | None = None, per_step=32):
    """Runs Newton-Schur (assemble, GMRES with restart-residual logging, recovery/update)
    through the C entry points and keeps, for every Newton step, a copy of the condensed
    tangent and the logged residuals.  u and beta advance in place.  Returns the list of
    (bsr_vals, samples) and the residual history."""
    lin = lin if lin is not None else B.solve_opts()
    data = []
    rn0 = None
    hist = []
    for _ in range(max_newton):
        A, rhs, rn = B.vms_condense_assemble(ctx, u, beta, Re, dt, u_prev, body)
        rnv = float(rn.item())
        hist.append(rnv)
        if rn0 is None:
            rn0 = rnv
        if rnv <= tol * rn0:
            break
        log = torch.zeros((per_step, ctx.n_nodes, 4), dtype=torch.float32, device=ctx.device)
        lin.log_residuals = log.data_ptr()
        lin.log_max = per_step
        du = ctx.new_vec()
        _, info = B.vms_gmres_solve(ctx, A, rhs, du, lin)
        lin.log_residuals = None
        lin.log_max = 0
        data.append((A, log[:max(1, info.logged)].contiguous()))
        B.vms_recover_update(ctx, u, beta, du, Re, dt, u_prev, body)
    return data, hist
