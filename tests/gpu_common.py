"""Helpers shared by the GPU tests: contexts from workload meshes, block-CSR
to scipy conversion, seeded random states.  (Imported by tests only.)"""
import numpy as np
import scipy.sparse as sp
import torch

DEV = "cuda:0"


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def make_context(B, mesh, dirichlet_dofs, precision=0, max_restart=50, basis_fp64=False):
    return B.Context(to_dev(mesh.xyz), to_dev(mesh.tets.astype(np.int32)),
                     to_dev(np.asarray(dirichlet_dofs, dtype=np.int32)), precision=precision,
                     max_restart=max_restart, basis_fp64=basis_fp64)


def bsr_to_csr(ctx, vals):
    """Scalar CSR (4 n_nodes square) of a block-CSR value tensor [nb, 16]."""
    rowptr, colidx, _ = ctx.bsr_pattern()
    v = vals.detach().double().cpu().numpy().reshape(-1, 4, 4)
    brow = np.repeat(np.arange(ctx.n_nodes), np.diff(rowptr))
    rows = (4 * brow[:, None, None] + np.arange(4)[None, :, None]).repeat(4, axis=2)
    cols = (4 * colidx[:, None, None] + np.arange(4)[None, None, :]).repeat(4, axis=1)
    n = 4 * ctx.n_nodes
    return sp.csr_matrix((v.ravel(), (rows.ravel(), cols.ravel())), shape=(n, n))


def random_state(mesh, seed, beta_scale=0.1, vel_scale=1.0):
    rng = np.random.default_rng(seed)
    u = vel_scale * rng.standard_normal((mesh.n_nodes, 4))
    up = u + 0.1 * rng.standard_normal((mesh.n_nodes, 4))
    beta = beta_scale * rng.standard_normal((mesh.n_elems, 3))
    body = rng.standard_normal((mesh.n_nodes, 3))
    return u, up, beta, body


def rel_fro(a, b):
    a = a.toarray() if sp.issparse(a) else np.asarray(a)
    b = b.toarray() if sp.issparse(b) else np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def sparse_rel_fro(A, B):
    D = (A - B)
    return float(sp.linalg.norm(D) / sp.linalg.norm(B))
