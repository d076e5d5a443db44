"""Full-size parity on the 64^3 jittered cube (1,572,864 tets, 274,625 nodes), through the C ABI.

* Condensed tangent and rhs (vms_condense_assemble) on a seeded sample of 1,000 block rows:
  the oracle (quadrature element, LU condensation, CSR assembly, Dirichlet elimination) is
  run on every element touching a sampled node, so the sampled rows are complete; GPU rows
  against oracle rows, norm-wise over the sample: FP64 1e-12, mixed 1e-5.  The state is the
  Ethier-Steinman field at t = 0 with a perturbed previous velocity and random fine scales, so
  every term of the residual and tangent (transient ones included) is exercised.
* vms_bsr_spmv on the GPU's own full-size matrix against a host product: at this size the
  SpMV grid exceeds 2,048 workgroups and takes its linear row order.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import vms as O
from oracle.element import element_residual_tangent
from workloads import build_workload
from tests.gpu_common import DEV, make_context, to_dev

pytestmark = pytest.mark.gpu


def _state(m, u0, seed):
    rng = np.random.default_rng(seed)
    u_prev = u0 + 0.05 * rng.standard_normal(u0.shape)
    beta = 0.01 * rng.standard_normal((m.n_elems, 3))
    return u_prev, beta


def _gpu_rows(ctx, vals, nodes):
    """Sampled block rows of the GPU matrix as a sparse [4 len(nodes), 4 n_nodes] matrix."""
    rowptr, colidx, _ = ctx.bsr_pattern()
    v = vals.detach().double().cpu().numpy().reshape(-1, 4, 4)
    rows, cols, data = [], [], []
    for k, i in enumerate(nodes):
        for p in range(rowptr[i], rowptr[i + 1]):
            r = 4 * k + np.arange(4)[:, None].repeat(4, 1)
            c = 4 * colidx[p] + np.arange(4)[None, :].repeat(4, 0)
            rows.append(r.ravel()); cols.append(c.ravel()); data.append(v[p].ravel())
    return sp.csr_matrix((np.concatenate(data), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(4 * len(nodes), 4 * ctx.n_nodes))


def test_es64_sampled_block_rows_against_oracle(vms_lib):
    B = vms_lib
    cfg, m, u0, beta0, bc = build_workload("es64")
    assert m.n_elems == 1_572_864
    u_prev, beta = _state(m, u0, seed=21)
    rng = np.random.default_rng(22)
    nodes = np.sort(rng.choice(m.n_nodes, size=1000, replace=False))
    patch = np.nonzero(np.isin(m.tets, nodes).any(axis=1))[0]
    nu, dt = 1.0 / cfg.re, cfg.dt
    print(f"es64 sampled rows: {len(nodes)} nodes, {len(patch)} patch elements", flush=True)
    R, K = element_residual_tangent(m.xyz, m.tets[patch], u0, beta[patch], nu, dt, u_prev, None)
    Ks, Rs = O.condense(R, K)
    A_ref = O.assemble_matrix(m.tets[patch], m.n_nodes, Ks, bc.dofs).tocsr()
    b_ref = -O.assemble_vector(m.tets[patch], m.n_nodes, Rs)
    b_ref[bc.dofs] = 0.0
    dof_rows = (4 * nodes[:, None] + np.arange(4)[None, :]).ravel()
    A_ref_rows = A_ref[dof_rows]
    b_ref_rows = b_ref[dof_rows]
    for prec, tol in ((B.VMS_FP64, 1e-12), (B.VMS_MIXED, 1e-5)):
        ctx = make_context(B, m, bc.dofs, prec)
        A, rhs, _ = B.vms_condense_assemble(ctx, to_dev(u0), to_dev(beta), cfg.re, dt, to_dev(u_prev))
        G = _gpu_rows(ctx, A, nodes)
        ea = sp.linalg.norm(G - A_ref_rows) / sp.linalg.norm(A_ref_rows)
        rb = rhs.cpu().numpy().reshape(-1)[dof_rows]
        eb = np.linalg.norm(rb - b_ref_rows) / np.linalg.norm(b_ref_rows)
        print(f"precision {prec}: sampled K* rows {ea:.2e}, rhs rows {eb:.2e}")
        assert ea <= tol and eb <= (1e-12 if prec == B.VMS_FP64 else 1e-12), (ea, eb)
        ctx.close()
        del A, rhs
        torch.cuda.empty_cache()


def test_es64_spmv_linear_row_order(vms_lib):
    B = vms_lib
    cfg, m, u0, beta0, bc = build_workload("es64")
    rng = np.random.default_rng(23)
    for prec, tol in ((B.VMS_FP64, 1e-14), (B.VMS_MIXED, 1e-6)):
        ctx = make_context(B, m, bc.dofs, prec)
        assert (8 * ctx.n_nodes + 255) // 256 > 2048            # SpMV grid: linear row order
        A, _, _ = B.vms_condense_assemble(ctx, to_dev(u0), to_dev(beta0), cfg.re, cfg.dt, to_dev(u0))
        x = torch.from_numpy(rng.standard_normal((m.n_nodes, 4))).to(DEV).to(ctx.dtype).contiguous()
        y = B.vms_bsr_spmv(ctx, A, x).double().cpu().numpy()
        rowptr, colidx, _ = ctx.bsr_pattern()
        Ah = A.double().cpu().numpy().reshape(-1, 4, 4)
        xh = x.double().cpu().numpy()
        prod = np.einsum("kij,kj->ki", Ah, xh[colidx])
        y_ref = np.add.reduceat(prod, rowptr[:-1], axis=0)
        err = np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref)
        print(f"precision {prec}: SpMV relative error {err:.2e}")
        assert err <= tol
        ctx.close()
        del A, x
        torch.cuda.empty_cache()
