"""Regression tests of the Krylov solver and error paths, through the C ABI.

* A block-diagonal matrix on a 64^3 cavity mesh (274,625 nodes, so the Arnoldi update launch has
  more than 2,048 workgroups): with the block-Jacobi preconditioner and the constant-pressure
  coarse correction, A P = I + (A z) z^T / (z^T A z) has the two eigenvalues 1 and 2, so the
  Krylov space closes at its second vector.  The stop is found by the update launch of step 1,
  whose other workgroups must still write q_1: the solve must end in that first cycle with the
  direct solution (per-block solves on the host).
* Deliberately bad learned weights (Delta = -e_0 e_0^T on every node: P_i drops each node's
  first component, so A P is singular) on a mixed context: the solver must give up the learned
  blocks after half of max_iters and converge with block-Jacobi within max_iters.
* The two refinement modes of the mixed solve reach the FP64 tolerance.
* A zero diagonal block: the preconditioner setup counts it (vms_solve_info.singular_blocks).
* NaN in the state: vms_newton_step returns VMS_ENONFINITE.
"""
import numpy as np
import pytest
import torch

from workloads import cavity_mesh, cavity_bc, apply_dirichlet, build_workload
from tests.gpu_common import DEV, bsr_to_csr, make_context, to_dev

pytestmark = pytest.mark.gpu


def _block_diagonal_system(ctx, seed):
    rowptr, colidx, diagpos = ctx.bsr_pattern()
    rng = np.random.default_rng(seed)
    n = ctx.n_nodes
    D = 0.1 * rng.standard_normal((n, 4, 4)) + np.eye(4)[None] * (2.0 + rng.random((n, 1, 1)))
    vals = np.zeros((ctx.nb, 16))
    vals[diagpos] = D.reshape(n, 16)
    vals = torch.from_numpy(vals).to(DEV).to(ctx.dtype).contiguous()
    Dm = vals[torch.from_numpy(diagpos.astype(np.int64)).to(DEV)].double().cpu().numpy().reshape(n, 4, 4)
    b = rng.standard_normal((n, 4))
    x_ref = np.linalg.solve(Dm, b[:, :, None])[:, :, 0]
    return vals, b, x_ref


@pytest.mark.parametrize("precision", [0, 1])
def test_invariant_krylov_space_on_a_large_grid(vms_lib, precision):
    B = vms_lib
    m = cavity_mesh(64)
    bc = cavity_bc(m)
    print(f"invariant-space regression: cavity 64^3 mesh, {m.n_nodes} nodes, precision {precision}", flush=True)
    ctx = make_context(B, m, bc.dofs, precision)
    # update launch: more than 2048 workgroups (from 131,072 nodes on, each XCD's eighth is the
    # rows of the dots' 8 of 64 chunks, two rows per thread)
    rows_per_xcd = 4 * -(-ctx.n_nodes // 64) * 8
    assert 8 * -(-rows_per_xcd // 512) > 2048
    vals, b, x_ref = _block_diagonal_system(ctx, seed=11 + precision)
    x = ctx.new_vec()
    rc, info = B.vms_gmres_solve(ctx, vals, to_dev(b), x, B.solve_opts(restart=50, rtol=1e-10, max_iters=400))
    err = np.linalg.norm(x.cpu().numpy() - x_ref) / np.linalg.norm(x_ref)
    print(f"iters {info.iters}, cycles {info.restarts}, refinements {info.refinements}, "
          f"true residual {info.true_rel_res:.2e}, error {err:.2e}")
    assert rc == B.VMS_OK and info.true_rel_res <= 1e-10
    if precision == 0:
        assert info.restarts == 1 and info.iters == 2
    else:
        # every FP32 sweep closes after a few vectors (the FP32 dot products decide the closing);
        # the FP64 refinement needs a few sweeps
        assert info.iters <= 4 * info.refinements
    assert err <= 1e-9


def _cavity8_system(B, precision, re=100.0):
    m = cavity_mesh(8)
    bc = cavity_bc(m)
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    ctx = make_context(B, m, bc.dofs, precision)
    A, rhs, _ = B.vms_condense_assemble(ctx, to_dev(u), to_dev(np.zeros((m.n_elems, 3))), re)
    return ctx, A, rhs


def test_bad_learned_weights_fall_back_in_mixed_precision(vms_lib):
    B = vms_lib
    ctx, A, rhs = _cavity8_system(B, B.VMS_MIXED)
    w = torch.zeros(B.PC_NWEIGHTS, dtype=torch.float32, device=DEV)
    w[-16] = -1.0                          # b2: Delta[0][0] = -1 on every node
    x = ctx.new_vec()
    rc, info = B.vms_gmres_solve(ctx, A, rhs, x, B.solve_opts(restart=50, rtol=1e-8, max_iters=4000,
                                                              pc=B.VMS_PC_LEARNED, pc_weights=w))
    print(f"bad weights: iters {info.iters}, fell back {info.fell_back_to_bj}, residual {info.true_rel_res:.2e}")
    assert rc == B.VMS_OK and info.fell_back_to_bj == 1
    assert info.true_rel_res <= 1e-8 and info.iters <= 4000
    # the same system with plain block-Jacobi, for scale: the fallback adds at most half the budget
    x2 = ctx.new_vec()
    _, info2 = B.vms_gmres_solve(ctx, A, rhs, x2, B.solve_opts(restart=50, rtol=1e-8, max_iters=4000))
    assert info.iters <= 2000 + 2 * info2.iters + 100


@pytest.mark.parametrize("inner_rtol", [0.0, 1e-4, 0.1])
def test_mixed_refinement_modes(vms_lib, inner_rtol):
    """Mixed GMRES with every cycle restarted from the FP64 residual (inner_rtol 0) and with
    FP32 sweeps to a tolerance: both reach rtol by the FP64 residual of the FP32-stored matrix
    (computed here on the host); per-cycle refinement counts one sweep per cycle."""
    B = vms_lib
    ctx, A, rhs = _cavity8_system(B, B.VMS_MIXED)
    x = ctx.new_vec()
    rc, info = B.vms_gmres_solve(ctx, A, rhs, x, B.solve_opts(restart=30, rtol=1e-10, max_iters=20000,
                                                              inner_rtol=inner_rtol, refine_max=1000))
    Am = bsr_to_csr(ctx, A)                  # the FP32-stored matrix, exactly, in FP64
    xs = x.cpu().numpy().ravel()
    bs = rhs.cpu().numpy().ravel()
    rel = np.linalg.norm(bs - Am @ xs) / np.linalg.norm(bs)
    print(f"inner_rtol {inner_rtol}: iters {info.iters}, cycles {info.restarts}, sweeps {info.refinements}, "
          f"residual {rel:.2e}")
    assert rc == B.VMS_OK and rel <= 1.01e-10 and info.true_rel_res <= 1e-10
    if inner_rtol == 0.0:
        assert info.refinements == info.restarts
    else:
        assert 1 <= info.refinements <= info.restarts


def test_singular_diagonal_block_is_reported(vms_lib):
    B = vms_lib
    m = cavity_mesh(8)
    bc = cavity_bc(m)
    fixed = np.unique(bc.dofs // 4)
    free = np.setdiff1d(np.arange(m.n_nodes), fixed)
    node = int(free[len(free) // 3])                 # a node without Dirichlet dofs
    for precision in (B.VMS_FP64, B.VMS_MIXED):
        ctx, A, rhs = _cavity8_system(B, precision)
        _, _, diagpos = ctx.bsr_pattern()
        # a clean matrix reports none
        _, info = B.vms_gmres_solve(ctx, A, rhs, ctx.new_vec(), B.solve_opts(restart=50, rtol=1e-8, max_iters=2000))
        assert info.singular_blocks == 0
        A[int(diagpos[node])] = 0.0
        _, info = B.vms_gmres_solve(ctx, A, rhs, ctx.new_vec(), B.solve_opts(restart=50, rtol=1e-8, max_iters=200),
                                    allow_noconv=True)
        assert info.singular_blocks == 1, info.singular_blocks


def test_nan_state_is_reported(vms_lib):
    B = vms_lib
    m = cavity_mesh(4)
    bc = cavity_bc(m)
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    interior = int(np.argmin(np.linalg.norm(m.xyz - 0.5, axis=1)))
    u[interior, 0] = np.nan
    ctx = make_context(B, m, bc.dofs, B.VMS_FP64)
    with pytest.raises(B.VmsError) as ei:
        B.vms_newton_step(ctx, to_dev(u), to_dev(np.zeros((m.n_elems, 3))), 10.0)
    assert ei.value.code == B.VMS_ENONFINITE
    # the residual norm alone is non-finite too, and vms_gmres_solve rejects a NaN right-hand side
    _, rn = B.vms_residual(ctx, to_dev(u), to_dev(np.zeros((m.n_elems, 3))), 10.0)
    assert not np.isfinite(float(rn.item()))
    u2 = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u2, bc)
    A, rhs, _ = B.vms_condense_assemble(ctx, to_dev(u2), to_dev(np.zeros((m.n_elems, 3))), 10.0)
    rhs[interior, 1] = float("nan")
    with pytest.raises(B.VmsError) as ei:
        B.vms_gmres_solve(ctx, A, rhs, ctx.new_vec(), B.solve_opts())
    assert ei.value.code == B.VMS_ENONFINITE
