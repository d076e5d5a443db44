"""ORACLE (test infrastructure): learned block-Jacobi correction, FP64.

The paper leaves the Krylov preconditioner unspecified (Section 6: PETSc
KSP, tolerance 1e-12, at most 50 iterations).  The build adds a learned
correction to 4x4 block-Jacobi; this module is its plain definition:

  features x_i (25) of node i, from the condensed tangent A (4x4 blocks):
      D_i / ||D_i||_F                      (16, row-major diagonal block)
      log ||D_i||_F                        (1)
      log(1 + sum_{j != i} ||A_ij[r, :]||_1 / |D_i[r, r]|),  r = 0..3     (4)
      Dirichlet flag of dof r,  r = 0..3   (4)
  MLP   h = tanh(W1 x + b1)  (64),  y = W2 h + b2  (16)  ->  Delta_i (4x4 row-major)
  mask  Delta_i[r, :] = Delta_i[:, r] = 0 for every Dirichlet dof r of node i
  P_i = D_i^-1 (I + Delta_i)
  loss  L = mean over samples of ||r - A P r||^2 / ||r||^2
  Adam  (beta1 0.9, beta2 0.999, eps 1e-8), bias-corrected.
Weights are packed as [W1 (64x25 row-major), b1 (64), W2 (16x64), b2 (16)].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

N_IN = 25
N_HID = 64
N_OUT = 16
N_WEIGHTS = N_HID * N_IN + N_HID + N_OUT * N_HID + N_OUT


def unpack(wts):
    o = 0
    W1 = wts[o:o + N_HID * N_IN].reshape(N_HID, N_IN); o += N_HID * N_IN
    b1 = wts[o:o + N_HID]; o += N_HID
    W2 = wts[o:o + N_OUT * N_HID].reshape(N_OUT, N_HID); o += N_OUT * N_HID
    b2 = wts[o:o + N_OUT]
    return W1, b1, W2, b2


def pack(W1, b1, W2, b2):
    return np.concatenate([W1.ravel(), b1.ravel(), W2.ravel(), b2.ravel()])


def node_blocks(A, n_nodes):
    """Diagonal blocks D [n, 4, 4] and per-row off-diagonal absolute row sums [n, 4]."""
    Acoo = A.tocoo()
    rn, cn = Acoo.row // 4, Acoo.col // 4
    D = np.zeros((n_nodes, 4, 4))
    diag = rn == cn
    np.add.at(D, (rn[diag], Acoo.row[diag] % 4, Acoo.col[diag] % 4), Acoo.data[diag])
    off = np.zeros((n_nodes, 4))
    np.add.at(off, (rn[~diag], Acoo.row[~diag] % 4), np.abs(Acoo.data[~diag]))
    return D, off


def features(A, n_nodes, dirichlet_dofs):
    D, off = node_blocks(A, n_nodes)
    fro = np.sqrt(np.sum(D ** 2, axis=(1, 2)))
    dflag = np.zeros(4 * n_nodes)
    dflag[dirichlet_dofs] = 1.0
    dd = np.abs(np.diagonal(D, axis1=1, axis2=2))
    x = np.concatenate([(D / fro[:, None, None]).reshape(n_nodes, 16),
                        np.log(fro)[:, None],
                        np.log1p(off / dd),
                        dflag.reshape(n_nodes, 4)], axis=1)
    return x, D


def dirichlet_mask(n_nodes, dirichlet_dofs):
    """[n, 4, 4] with 0 on the rows and columns of Dirichlet dofs, else 1."""
    free = np.ones(4 * n_nodes)
    free[dirichlet_dofs] = 0.0
    f = free.reshape(n_nodes, 4)
    return f[:, :, None] * f[:, None, :]


def mlp_forward(wts, x):
    W1, b1, W2, b2 = unpack(wts)
    h = np.tanh(x @ W1.T + b1)
    y = h @ W2.T + b2
    return y, h


def preconditioner_blocks(wts, x, D, mask):
    """P_i = D_i^-1 (I + Delta_i) [n, 4, 4]."""
    y, _ = mlp_forward(wts, x)
    delta = y.reshape(-1, 4, 4) * mask
    return np.linalg.inv(D) @ (np.eye(4)[None] + delta)


def apply_blocks(P, v):
    return np.einsum("nij,nj->ni", P, v.reshape(-1, 4)).ravel()


def loss_and_grad(wts, A, x, D, mask, rs):
    """Mean loss over the residual samples rs [S, 4n] and its gradient."""
    W1, b1, W2, b2 = unpack(wts)
    y, h = mlp_forward(wts, x)
    Dinv = np.linalg.inv(D)
    P = Dinv @ (np.eye(4)[None] + y.reshape(-1, 4, 4) * mask)
    At = A.T.tocsr()
    loss = 0.0
    gdelta = np.zeros_like(P)
    for r in rs:
        rr = r @ r
        s = apply_blocks(P, r)
        e = r - A @ s
        loss += (e @ e) / rr
        gs = (-2.0 / rr) * (At @ e)                       # dL/ds
        gP = gs.reshape(-1, 4)[:, :, None] * r.reshape(-1, 4)[:, None, :]
        gdelta += np.transpose(Dinv, (0, 2, 1)) @ gP      # D^-T dL/dP
    S = len(rs)
    loss /= S
    gy = (gdelta * mask).reshape(-1, 16) / S
    gW2 = gy.T @ h
    gb2 = gy.sum(axis=0)
    gz = (gy @ W2) * (1.0 - h ** 2)
    gW1 = gz.T @ x
    gb1 = gz.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2)


def init_weights(seed=1):
    """Glorot-uniform first layer, zero output layer (the network starts as
    exact block-Jacobi)."""
    rng = np.random.default_rng(seed)
    lim = np.sqrt(6.0 / (N_IN + N_HID))
    W1 = rng.uniform(-lim, lim, size=(N_HID, N_IN))
    return pack(W1, np.zeros(N_HID), np.zeros((N_OUT, N_HID)), np.zeros(N_OUT))


def adam_step(wts, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  Returns new (wts, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mhat = m / (1 - b1 ** t)
    vhat = v / (1 - b2 ** t)
    return wts - lr * mhat / (np.sqrt(vhat) + eps), m, v


def as_sparse(A):
    return A if sp.issparse(A) else sp.csr_matrix(A)
