"""Deflated restarting (GMRES-DR: Morgan, SIAM J. Sci. Comput. 24 (2002)) through the C ABI.

Two condensed systems on which restarted GMRES loses most of its progress at every restart:
the first Newton tangent of the lid-driven cavity on an 8^3 mesh at Re 400 (one pressure dof
pinned, coarse pressure correction on), and of the backward-facing step with (1, 2, 1) cells
per unit length at Re 50 (open outlet, no pressure pin).  With and without deflation, FP64 and
mixed: the true residual of the returned x, computed on the host with the stored matrix, meets
rtol; x agrees with scipy's direct solve; the deflated solve restarted several times (so the
kept basis, its Hessenberg block and the prefix transform of the Givens chain were exercised)
and took fewer Arnoldi steps.  On the backward-facing step, whose preconditioner is plain
block-Jacobi (no pressure pin, so no coarse correction), the FP64 steps and cycles match the
oracle's GMRES-DR (oracle/gmres_dr.py) run on the same stored matrix.  The invalid option
combinations are refused.  A transient backward-facing-step Newton solve in mixed precision
exercises the safeguard (deflated cycles that raise the true residual are undone) and shows the
FP64 basis needs none.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import vms as O
from oracle.gmres_dr import gmres_dr

from workloads import backward_facing_step, bfs_bc, cavity_bc, cavity_mesh, apply_dirichlet
from tests.gpu_common import bsr_to_csr, make_context, to_dev

pytestmark = pytest.mark.gpu

# restart length, vectors kept, bound on (deflated steps) / (plain steps)
CASES = {"cavity8": (20, 6, 0.9), "bfs121": (30, 10, 0.5)}


def _system(B, case, precision, basis_fp64=False):
    if case == "cavity8":
        m = cavity_mesh(8)
        bc = cavity_bc(m)
        re = 400.0
    else:
        m = backward_facing_step(1, 2, 1)
        bc = bfs_bc(m)
        re = 50.0
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    ctx = make_context(B, m, bc.dofs, precision, basis_fp64=basis_fp64)
    A, rhs, _ = B.vms_condense_assemble(ctx, to_dev(u), to_dev(np.zeros((m.n_elems, 3))), re)
    return ctx, A, rhs


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("case", sorted(CASES))
def test_deflated_restarts_reach_the_direct_solution_in_fewer_steps(vms_lib, case, precision):
    B = vms_lib
    restart, k, ratio = CASES[case]
    print(f"deflation: {case}, precision {precision}, restart {restart}, k {k}", flush=True)
    ctx, A, rhs = _system(B, case, precision)
    Am = bsr_to_csr(ctx, A)
    bs = rhs.cpu().numpy().ravel()
    xd = spla.spsolve(Am.tocsc(), bs)
    infos = {}
    for kk in (0, k):
        x = ctx.new_vec()
        rc, info = B.vms_gmres_solve(ctx, A, rhs, x, B.solve_opts(restart=restart, rtol=1e-10, max_iters=20000,
                                                                  deflate=kk))
        xs = x.cpu().numpy().ravel()
        rel = np.linalg.norm(bs - Am @ xs) / np.linalg.norm(bs)
        err = np.linalg.norm(xs - xd) / np.linalg.norm(xd)
        print(f"  deflate {kk}: rc {rc}, steps {info.iters}, cycles {info.restarts}, residual {rel:.2e}, "
              f"error vs direct {err:.2e}", flush=True)
        assert rc == B.VMS_OK and info.true_rel_res <= 1e-10 and rel <= 1.01e-10
        assert err <= 1e-6
        infos[kk] = info
    assert infos[k].restarts >= 3
    assert infos[k].iters <= ratio * infos[0].iters


@pytest.mark.parametrize("restart,k", [(30, 10), (20, 5), (40, 16), (50, 24)])
def test_deflated_steps_match_the_oracle(vms_lib, restart, k):
    B = vms_lib
    print(f"deflation parity: bfs121 FP64, restart {restart}, k {k}", flush=True)
    ctx, A, rhs = _system(B, "bfs121", B.VMS_FP64)
    Am = bsr_to_csr(ctx, A)
    bs = rhs.cpu().numpy().ravel()
    ref = gmres_dr(Am, bs, restart=restart, k=k, rtol=1e-10, max_iters=20000,
                   Minv_blocks=O.block_jacobi_inverse(Am, ctx.n_nodes))
    x = ctx.new_vec()
    rc, info = B.vms_gmres_solve(ctx, A, rhs, x, B.solve_opts(restart=restart, rtol=1e-10, max_iters=20000,
                                                              deflate=k))
    print(f"  GPU {info.iters} steps / {info.restarts} cycles; oracle {ref.iters} / {ref.restarts}")
    assert rc == B.VMS_OK and ref.converged
    # rounding (the device's Gram-Schmidt and reduction orders) may move the stop by a step or two
    assert abs(info.iters - ref.iters) <= max(3, 0.01 * ref.iters)
    assert abs(info.restarts - ref.restarts) <= 1
    xs = x.cpu().numpy().ravel()
    assert np.linalg.norm(xs - ref.x) <= 1e-7 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("k", [0, 10])
def test_fp64_basis_on_a_mixed_context(vms_lib, k):
    """Mixed context, FP64 Krylov basis: FP64 GMRES (cycles on the FP64 residual, no refinement
    sweeps) on the FP32-stored matrix.  The oracle runs on that matrix exactly; the device's
    A P and preconditioner blocks are FP32-rounded, so the steps may differ by a few."""
    B = vms_lib
    print(f"FP64 basis on a mixed context: bfs121, restart 30, k {k}", flush=True)
    ctx, A, rhs = _system(B, "bfs121", B.VMS_MIXED, basis_fp64=True)
    Am = bsr_to_csr(ctx, A)
    bs = rhs.cpu().numpy().ravel()
    ref = gmres_dr(Am, bs, restart=30, k=k, rtol=1e-10, max_iters=20000,
                   Minv_blocks=O.block_jacobi_inverse(Am, ctx.n_nodes))
    x = ctx.new_vec()
    rc, info = B.vms_gmres_solve(ctx, A, rhs, x, B.solve_opts(restart=30, rtol=1e-10, max_iters=20000, deflate=k,
                                                              basis_fp64=1))
    xs = x.cpu().numpy().ravel()
    rel = np.linalg.norm(bs - Am @ xs) / np.linalg.norm(bs)
    print(f"  GPU {info.iters} steps / {info.restarts} cycles, residual {rel:.2e}; oracle {ref.iters} / {ref.restarts}")
    assert rc == B.VMS_OK and rel <= 1.01e-10 and info.refinements == 0 and info.deflation_stopped == 0
    assert abs(info.iters - ref.iters) <= max(5, 0.03 * ref.iters)


def test_deflation_options_are_checked(vms_lib):
    B = vms_lib
    ctx, A, rhs = _system(B, "cavity8", B.VMS_FP64)
    for opts in (dict(restart=20, deflate=19), dict(restart=50, deflate=33), dict(restart=20, deflate=-1)):
        with pytest.raises(B.VmsError) as e:
            B.vms_gmres_solve(ctx, A, rhs, ctx.new_vec(), B.solve_opts(rtol=1e-8, **opts))
        assert e.value.code == B.VMS_EINVAL, opts
    mctx, mA, mrhs = _system(B, "cavity8", B.VMS_MIXED)
    with pytest.raises(B.VmsError) as e:
        B.vms_gmres_solve(mctx, mA, mrhs, mctx.new_vec(), B.solve_opts(restart=20, deflate=5, inner_rtol=1e-4))
    assert e.value.code == B.VMS_EINVAL
    # an FP64 basis is allocated by vms_create only: a mixed context created without one refuses
    # it, and an FP64 context ignores the option
    with pytest.raises(B.VmsError) as e:
        B.vms_gmres_solve(mctx, mA, mrhs, mctx.new_vec(), B.solve_opts(restart=20, deflate=5, basis_fp64=1))
    assert e.value.code == B.VMS_EINVAL
    rc, info = B.vms_gmres_solve(ctx, A, rhs, ctx.new_vec(), B.solve_opts(restart=20, rtol=1e-8, basis_fp64=1))
    assert rc == B.VMS_OK and info.true_rel_res <= 1e-8
    # the largest kept count a restart length allows
    x = ctx.new_vec()
    rc, info = B.vms_gmres_solve(ctx, A, rhs, x, B.solve_opts(restart=20, deflate=18, rtol=1e-10, max_iters=20000))
    print(f"deflate 18 of 20: rc {rc}, steps {info.iters}, cycles {info.restarts}")
    assert rc == B.VMS_OK and info.true_rel_res <= 1e-10


def test_safeguard_undoes_deflated_cycles_that_raise_the_residual(vms_lib):
    """First backward-Euler step of the backward-facing step (1, 2, 1) at Re 800, dt 0.05, from
    rest, mixed precision, deterministic context (bitwise reproducible assemblies and solves).
    With an FP32 basis, deflated cycles of some Newton systems raise the true residual (the
    kept block drifts from the FP32-rounded basis): each is undone and that solve continues with
    plain restarts (deflation_stopped), and the Newton solve still reaches 1e-8, by the
    oracle's FP64 residual of the returned state.  With an FP64 basis no cycle is undone."""
    from paper_0809_4802_amd import driver
    import torch
    B = vms_lib
    m = backward_facing_step(1, 2, 1)
    bc = bfs_bc(m)
    u0 = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u0, bc)
    ctx = B.Context(to_dev(m.xyz), to_dev(m.tets.astype(np.int32)), to_dev(np.asarray(bc.dofs, dtype=np.int32)),
                    precision=B.VMS_MIXED, deterministic=True, basis_fp64=True)
    stopped = {}
    for b64 in (0, 1):
        print(f"safeguard: bfs121 transient Re 800, mixed, basis_fp64 {b64}", flush=True)
        u = to_dev(u0)
        beta = torch.zeros((m.n_elems, 3), dtype=torch.float64, device=u.device)
        u_prev = torch.zeros_like(u)
        lin = B.solve_opts(restart=50, rtol=1e-9, max_iters=400000, deflate=10, basis_fp64=b64)
        r = driver.newton_solve(ctx, u, beta, 800.0, 0.05, u_prev, None, tol=1e-8, lin=lin, forcing="ew")
        stopped[b64] = [d["deflation_stopped"] for d in r.lin]
        print(f"  Newton {len(r.rnorms) - 1}, GMRES {[d['iters'] for d in r.lin]}, undone {stopped[b64]}")
        assert r.converged
        prob = O.Problem(m.xyz, m.tets, bc.dofs, nu=1.0 / 800.0, dt=0.05, u_prev=np.zeros((m.n_nodes, 4)))
        rn = O.residual_norm_at(prob, u.cpu().numpy(), beta.cpu().numpy())
        assert rn <= 1.01e-8 * r.rnorms[0], (rn, r.rnorms[0])
    assert sum(stopped[0]) >= 1
    assert sum(stopped[1]) == 0


def test_learned_fallback_drops_the_kept_basis(vms_lib):
    """Deliberately bad learned weights (Delta = -e_0 e_0^T on every node: a singular A P) with
    deflated restarts, mixed context: the solve gives up the learned blocks after half of
    max_iters, and the kept basis, which belongs to the old operator, is dropped with them
    (the first cycle on block-Jacobi restarts plainly); it then converges to rtol with
    block-Jacobi, by the FP64 residual of the stored matrix.  (On the singular operator a
    deflated cycle may already have raised the residual, in which case the safeguard stopped
    deflation before the switch.)"""
    import torch
    B = vms_lib
    ctx, A, rhs = _system(B, "cavity8", B.VMS_MIXED)
    w = torch.zeros(B.PC_NWEIGHTS, dtype=torch.float32, device=A.device)
    w[-16] = -1.0                          # b2: Delta[0][0] = -1 on every node
    x = ctx.new_vec()
    rc, info = B.vms_gmres_solve(ctx, A, rhs, x, B.solve_opts(restart=20, rtol=1e-10, max_iters=4000, deflate=6,
                                                              pc=B.VMS_PC_LEARNED, pc_weights=w))
    Am = bsr_to_csr(ctx, A)
    bs = rhs.cpu().numpy().ravel()
    rel = np.linalg.norm(bs - Am @ x.cpu().numpy().ravel()) / np.linalg.norm(bs)
    print(f"bad weights + deflation: rc {rc}, steps {info.iters}, fell back {info.fell_back_to_bj}, "
          f"undone {info.deflation_stopped}, residual {rel:.2e}")
    assert rc == B.VMS_OK and info.fell_back_to_bj == 1 and rel <= 1.01e-10
    assert info.iters <= 4000
