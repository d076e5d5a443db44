"""Fixed-point (Picard) linearisation on the GPU, through the C ABI, against the oracle.

The tangent holds the advecting velocity at the current iterate (the alternative to
Newton's consistent linearisation that the introduction argues against); the residual is
unchanged.  Tolerances: FP64 1e-12 on element blocks and assembled matrices, mixed 1e-5;
one FP64 Picard step against the oracle's condensed Picard system (cross residual) and
recovery; a cavity solve converges linearly to the Newton solution.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import vms as O
from oracle.element import element_residual_tangent
from workloads import jitter_interior, kuhn_box, boundary_nodes, cavity_mesh, cavity_bc, apply_dirichlet
from tests.gpu_common import DEV, to_dev, make_context, bsr_to_csr, random_state, rel_fro

pytestmark = pytest.mark.gpu


def _mesh():
    m = jitter_interior(kuhn_box((4, 3, 5), (0, 0, 0), (1.0, 0.8, 1.3)), 0.2, 9)
    bnd = np.nonzero(boundary_nodes(m.tets, m.n_nodes))[0]
    dofs = np.unique(np.concatenate([(4 * bnd[:, None] + np.arange(3)).ravel(), [3]])).astype(np.int32)
    return m, dofs


def _picard_context(B, m, dofs, precision, full=False):
    ctx = B.Context(to_dev(m.xyz), to_dev(m.tets.astype(np.int32)), to_dev(dofs), precision=precision,
                    full_system=full)
    B.vms_set_linearization(ctx, B.VMS_LIN_PICARD)
    return ctx


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_picard_element_tangents_match_oracle(vms_lib, precision, tol):
    B = vms_lib
    m, dofs = _mesh()
    ctx = _picard_context(B, m, dofs, precision)
    u, up, beta, body = random_state(m, 31, beta_scale=0.2)
    Re, dt = 45.0, 0.03
    Ke, Rv = B.vms_element_tangents(ctx, to_dev(u), to_dev(beta), Re, dt, to_dev(up), to_dev(body))
    R_o, K_o = element_residual_tangent(m.xyz, m.tets, u, beta, 1 / Re, dt, up, body, picard=True)
    _, K_n = element_residual_tangent(m.xyz, m.tets, u, beta, 1 / Re, dt, up, body)
    ek = np.linalg.norm(Ke.cpu().numpy() - K_o, axis=(1, 2)) / np.linalg.norm(K_o, axis=(1, 2))
    er = np.linalg.norm(Rv.cpu().numpy() - R_o, axis=1) / np.linalg.norm(R_o, axis=1)
    assert ek.max() <= tol, ek.max()
    assert er.max() <= 1e-12, er.max()
    # the two tangents differ by far more than the tolerance (the flag is honoured)
    assert np.min(np.linalg.norm(K_n - K_o, axis=(1, 2)) / np.linalg.norm(K_o, axis=(1, 2))) > 100 * tol
    # and the switch goes back
    B.vms_set_linearization(ctx, B.VMS_LIN_NEWTON)
    Ke2, _ = B.vms_element_tangents(ctx, to_dev(u), to_dev(beta), Re, dt, to_dev(up), to_dev(body))
    assert np.max(np.linalg.norm(Ke2.cpu().numpy() - K_n, axis=(1, 2)) / np.linalg.norm(K_n, axis=(1, 2))) <= tol
    with pytest.raises(B.VmsError) as e:
        B.vms_set_linearization(ctx, 2)
    assert e.value.code == B.VMS_EINVAL


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_picard_condensed_and_uncondensed_assembly(vms_lib, precision, tol):
    from tests.test_gpu_full_newton import _to_oracle_layout
    B = vms_lib
    m, dofs = _mesh()
    ctx = _picard_context(B, m, dofs, precision, full=True)
    u, up, beta, body = random_state(m, 32, beta_scale=0.2)
    Re, dt = 45.0, 0.03
    prob = O.Problem(m.xyz, m.tets, dofs, nu=1 / Re, dt=dt, u_prev=up, body=body, picard=True)
    A_g, rhs_g, rn_g = B.vms_condense_assemble(ctx, to_dev(u), to_dev(beta), Re, dt, to_dev(up), to_dev(body))
    A_o, b_o, _, _ = O.condensed_system(prob, u, beta)
    assert sp.linalg.norm(bsr_to_csr(ctx, A_g) - A_o) <= tol * sp.linalg.norm(A_o)
    assert rel_fro(rhs_g.cpu().numpy().ravel(), b_o) <= 1e-12
    vals, rhs, _ = B.vms_full_assemble(ctx, to_dev(u), to_dev(beta), Re, dt, to_dev(up), to_dev(body))
    torch.cuda.synchronize()
    A, b, _, _ = _to_oracle_layout(ctx, vals, rhs, m)
    Af_o, bf_o = O.full_system(prob, u, beta)
    assert sp.linalg.norm(A - Af_o) <= tol * sp.linalg.norm(Af_o)
    assert np.linalg.norm(b - bf_o) <= 1e-12 * np.linalg.norm(bf_o)


def test_picard_step_matches_oracle(vms_lib):
    B = vms_lib
    m, dofs = _mesh()
    ctx = _picard_context(B, m, dofs, B.VMS_FP64)
    u, up, beta, body = random_state(m, 33, beta_scale=0.01, vel_scale=0.3)
    Re, dt = 60.0, 0.03
    ud, bd = to_dev(u), to_dev(beta)
    B.vms_newton_step(ctx, ud, bd, Re, dt, to_dev(up), to_dev(body), B.solve_opts(rtol=1e-13, max_iters=20000))
    prob = O.Problem(m.xyz, m.tets, dofs, nu=1 / Re, dt=dt, u_prev=up, body=body, picard=True)
    A_o, b_o, R, K = O.condensed_system(prob, u, beta)
    du = ud.cpu().numpy() - u
    assert np.linalg.norm(A_o @ du.ravel() - b_o) <= 1e-11 * np.linalg.norm(b_o)
    db_o = O.recover_fine(R, K, du.ravel()[O.element_coarse_dofs(m.tets)])
    assert rel_fro(bd.cpu().numpy() - beta, db_o) <= 1e-11


def test_picard_converges_linearly_to_the_newton_solution(vms_lib):
    """Cavity 4^3, Re 20, FP64: the Picard residual history follows the oracle's Picard
    iteration, decreases by a roughly constant factor, and ends at the Newton solution."""
    from paper_0809_4802_amd import driver
    B = vms_lib
    m = cavity_mesh(4)
    bc = cavity_bc(m)
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    Re = 20.0
    lin = B.solve_opts(rtol=1e-13, max_iters=20000)
    ctx = make_context(B, m, bc.dofs, B.VMS_FP64)
    un = to_dev(u)
    rn = driver.newton_solve(ctx, un, torch.zeros((m.n_elems, 3), dtype=torch.float64, device=DEV), Re,
                             tol=1e-11, lin=lin)
    B.vms_set_linearization(ctx, B.VMS_LIN_PICARD)
    up = to_dev(u)
    rp = driver.newton_solve(ctx, up, torch.zeros((m.n_elems, 3), dtype=torch.float64, device=DEV), Re,
                             tol=1e-11, lin=lin, max_newton=80)
    assert rp.converged and len(rp.rnorms) > len(rn.rnorms) + 2
    _, _, log_o = O.newton_solve(O.Problem(m.xyz, m.tets, bc.dofs, nu=1 / Re, picard=True), u,
                                 np.zeros((m.n_elems, 3)), tol=1e-11, max_newton=80)
    k = min(6, len(log_o.rnorms))
    assert np.allclose(rp.rnorms[:k], log_o.rnorms[:k], rtol=1e-6)
    r = np.array(rp.rnorms)
    rates = r[3:7] / r[2:6]
    assert np.all(rates < 0.5) and np.ptp(rates) < 0.1, rates
    assert rel_fro(up.cpu().numpy(), un.cpu().numpy()) <= 1e-9
