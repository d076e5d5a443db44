"""Training loop of the learned block-Jacobi correction (host orchestration).

Samples are residuals the method's own GMRES solves produce (the restart
residuals logged by vms_gmres_solve); every forward, backward and Adam step
runs in the library's kernels (vms_pc_train_step).
"""
from __future__ import annotations

import math
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
                        lin: B.SolveOpts | None = None, per_step=32, allow_noconv=False):
    """Runs Newton-Schur (assemble, GMRES with restart-residual logging, recovery/update)
    through the C entry points and keeps, for every Newton step, a copy of the condensed
    tangent and the logged residuals.  u and beta advance in place.  Returns the list of
    (bsr_vals, samples) and the residual history.  allow_noconv: a linear solve that misses
    its tolerance within lin.max_iters still contributes its system and residuals, and
    Newton continues from its iterate."""
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
        _, info = B.vms_gmres_solve(ctx, A, rhs, du, lin, allow_noconv=allow_noconv)
        lin.log_residuals = None
        lin.log_max = 0
        data.append((A, log[:max(1, info.logged)].contiguous()))
        B.vms_recover_update(ctx, u, beta, du, Re, dt, u_prev, body)
    return data, hist


def gmres_iterations(ctx: B.Context, A, b, weights, rtol=1e-4, max_iters=20000, restart=50):
    """Arnoldi steps GMRES(restart) needs on A x = b with the learned blocks (None: block-Jacobi)."""
    x = ctx.new_vec()
    opts = B.solve_opts(restart=restart, rtol=rtol, max_iters=max_iters,
                        pc=B.VMS_PC_LEARNED if weights is not None else B.VMS_PC_BLOCK_JACOBI,
                        pc_weights=weights)
    rc, info = B.vms_gmres_solve(ctx, A, b, x, opts, allow_noconv=True)
    if rc != B.VMS_OK or info.fell_back_to_bj:
        return max_iters
    return int(info.iters)


def train_validated(ctx: B.Context, data, val, steps=200, lr=3e-4, batch=8, seed=1, check_every=20,
                    val_rtol=1e-4, val_restart=50, val_max_iters=20000, min_gain=0.2, lr_decay="none"):
    """Trains on `data` and keeps the checkpoint with the fewest GMRES iterations on the
    held-out systems `val` (list of (bsr_vals, rhs)); plain block-Jacobi (the zero output
    layer) is one of the candidates, so the result is never worse on the validation set.
    A checkpoint replaces block-Jacobi only if it saves at least min_gain of its validation
    iterations: restarted GMRES counts scatter widely under small perturbations of the
    operator, so a smaller gain is not evidence that the correction helps.
    lr_decay: "none" keeps lr; "cosine" scales it by (1 + cos(pi (step - 1) / steps)) / 2.
    Returns (weights or None for block-Jacobi, report)."""
    if lr_decay not in ("none", "cosine"):
        raise ValueError(f"lr_decay must be 'none' or 'cosine', not {lr_decay!r}")
    def score(w, cap=val_max_iters):
        return sum(gmres_iterations(ctx, A, b, w, rtol=val_rtol, max_iters=cap, restart=val_restart) for A, b in val)

    base = score(None)
    cap = max(100, 2 * base // max(1, len(val)))      # a checkpoint slower than 2x block-Jacobi is out
    best_w, best = None, base
    report = {"val_iters_bj": base, "checkpoints": []}
    rng = np.random.default_rng(seed)
    w = init_weights(seed, ctx.device)
    state = torch.zeros(2 * B.PC_NWEIGHTS, dtype=torch.float32, device=ctx.device)
    loss = torch.zeros(1, dtype=torch.float32, device=ctx.device)
    for step in range(1, steps + 1):
        A, S = data[rng.integers(len(data))]
        k = min(batch, S.shape[0])
        idx = torch.from_numpy(rng.choice(S.shape[0], size=k, replace=False)).to(ctx.device)
        lr_t = lr * (0.5 * (1.0 + math.cos(math.pi * (step - 1) / steps)) if lr_decay == "cosine" else 1.0)
        B.vms_pc_train_step(ctx, A, S.index_select(0, idx).contiguous(), w, state, step, lr_t, None, loss)
        if step % check_every == 0:
            s = score(w, cap)
            report["checkpoints"].append({"step": step, "loss": float(loss.item()), "val_iters": s})
            if s < best and s <= (1.0 - min_gain) * base:
                best, best_w = s, w.clone()
    report["selected"] = "bj" if best_w is None else "learned"
    report["val_iters_selected"] = best
    return best_w, report


def train_select(ctx: B.Context, data, val, seeds=(1, 2, 3), **kw):
    """train_validated for each seed; keeps the weights with the fewest validation iterations.
    Returns (weights or None, report with one entry per seed)."""
    best_w, best, reports = None, None, []
    for seed in seeds:
        w, rep = train_validated(ctx, data, val, seed=seed, **kw)
        rep["seed"] = seed
        reports.append(rep)
        if best is None or rep["val_iters_selected"] < best:
            best, best_w = rep["val_iters_selected"], w
    return best_w, {"val_iters_bj": reports[0]["val_iters_bj"], "val_iters_selected": best,
                    "selected": "bj" if best_w is None else "learned", "runs": reports}
