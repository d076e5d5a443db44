"""Pins of the oracle's condensation, solves and Newton loop (not gpu).

  * a Newton-Schur step equals the brute-force Newton step on the full
    uncondensed system (block Gauss elimination is exact algebra, Section 5;
    the paper reports identical Newton-Schur and Newton-Raphson results,
    Section 6.1)
  * Newton converges quadratically (Abstract; Introduction)
  * restarted GMRES + block-Jacobi reaches the direct solution; the true
    residual is recomputed independently
  * Ethier-Steinman manufactured solution: velocity converges at close to
    second order and stays near the best (interpolation) error
"""
import numpy as np
import pytest

from oracle import vms
from oracle.errors import l2_errors
from workloads import (cavity_mesh, jittered_cube, cavity_bc, ethier_steinman_bc,
                       apply_dirichlet, es_velocity, es_pressure, ES_D)
from workloads.ethier_steinman import es_nodal


def cavity_problem(n, re):
    m = cavity_mesh(n)
    bc = cavity_bc(m)
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    return m, vms.Problem(m.xyz, m.tets, bc.dofs, nu=1.0 / re), u, np.zeros((m.n_elems, 3))


@pytest.mark.parametrize("re", [1.0, 100.0])
def test_schur_step_equals_full_newton_step_cavity(re):
    m, prob, u, beta = cavity_problem(4, re)
    for _ in range(2):               # from the initial guess and from a nonzero beta
        u1, b1, _, _ = vms.newton_schur_step(prob, u, beta)
        u2, b2 = vms.full_newton_step(prob, u, beta)
        assert np.max(np.abs(u1 - u2)) <= 1e-12 * np.max(np.abs(u2))
        assert np.max(np.abs(b1 - b2)) <= 1e-12 * np.max(np.abs(b2))
        u, beta = u1, b1


def test_schur_step_equals_full_newton_step_transient_jittered():
    m = jittered_cube(3, seed=2)
    nu_l = 2.0 / 50.0
    bc = ethier_steinman_bc(m, 0.02, nu_l)
    rng = np.random.default_rng(9)
    up = es_nodal(m.xyz, 0.0, nu_l)
    u = up.copy()
    apply_dirichlet(u, bc)
    beta = 0.01 * rng.standard_normal((m.n_elems, 3))
    body = rng.standard_normal((m.n_nodes, 3))
    prob = vms.Problem(m.xyz, m.tets, bc.dofs, nu=1 / 50.0, dt=0.02, u_prev=up, body=body)
    u1, b1, _, _ = vms.newton_schur_step(prob, u, beta)
    u2, b2 = vms.full_newton_step(prob, u, beta)
    assert np.max(np.abs(u1 - u2)) <= 1e-12 * np.max(np.abs(u2))
    assert np.max(np.abs(b1 - b2)) <= 1e-12 * np.max(np.abs(b2))


def test_newton_converges_quadratically():
    m, prob, u, beta = cavity_problem(4, 100.0)
    _, _, log = vms.newton_solve(prob, u, beta, tol=1e-12)
    r = np.array(log.rnorms)
    assert r[-1] <= 1e-12 * r[0]
    # ||R_{k+1}|| <= C ||R_k||^2 over the last steps above round-off
    k = [i for i in range(len(r) - 1) if r[i + 1] > 1e-13 * r[0]]
    assert len(k) >= 2
    ratios = [r[i + 1] / r[i] ** 2 for i in k[-2:]]
    assert max(ratios) < 50.0
    assert np.log(r[k[-1] + 1]) / np.log(r[k[-1]]) > 1.8


def test_gmres_block_jacobi_reaches_direct_solution():
    m, prob, u, beta = cavity_problem(4, 100.0)
    A, b, _, _ = vms.condensed_system(prob, u, beta)
    x_d = vms.solve_direct(A, b)
    res = vms.gmres(A, b, restart=50, rtol=1e-12, max_iters=5000,
                    Minv_blocks=vms.block_jacobi_inverse(A, m.n_nodes))
    assert res.converged
    true = np.linalg.norm(b - A @ res.x) / np.linalg.norm(b)
    assert true <= 1e-12
    cond = np.linalg.cond(A.toarray())
    assert np.linalg.norm(res.x - x_d) <= 10 * 1e-12 * cond * np.linalg.norm(x_d)
    # the cap is honoured and reported
    short = vms.gmres(A, b, restart=50, rtol=1e-12, max_iters=3,
                      Minv_blocks=vms.block_jacobi_inverse(A, m.n_nodes))
    assert not short.converged and short.iters == 3


def test_block_jacobi_blocks():
    m, prob, u, beta = cavity_problem(4, 10.0)
    A, _, _, _ = vms.condensed_system(prob, u, beta)
    Dinv = vms.block_jacobi_inverse(A, m.n_nodes)
    Ad = A.toarray()
    for i in (0, 31, 62, 124):
        D = Ad[4 * i:4 * i + 4, 4 * i:4 * i + 4]
        assert np.allclose(Dinv[i] @ D, np.eye(4), atol=1e-12)


def test_dirichlet_rows_and_pin():
    m, prob, u, beta = cavity_problem(4, 1.0)
    A, b, _, _ = vms.condensed_system(prob, u, beta)
    Ad = A.toarray()
    for d in prob.dirichlet_dofs[:20]:
        row = Ad[d].copy()
        col = Ad[:, d].copy()
        assert row[d] == 1.0 and col[d] == 1.0
        row[d] = 0
        col[d] = 0
        assert not row.any() and not col.any()
        assert b[d] == 0.0
    # the pressure block of a free node is negative (stabilisation), not zero
    free_p = [4 * i + 3 for i in range(m.n_nodes) if 4 * i + 3 not in set(prob.dirichlet_dofs)]
    assert np.all(np.diag(Ad)[free_p] < 0)


def _es_steady(n, re):
    nu = 1.0 / re
    nu_l = 2.0 * nu
    m = jittered_cube(n, seed=0)
    bc = ethier_steinman_bc(m, 0.0, nu_l)
    ex = es_nodal(m.xyz, 0.0, nu_l)
    body = 2.0 * nu * ES_D ** 2 * ex[:, :3]          # -2 nu lap(u) of the Beltrami field
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    prob = vms.Problem(m.xyz, m.tets, bc.dofs, nu=nu, body=body)
    us, _, _ = vms.newton_solve(prob, u, np.zeros((m.n_elems, 3)), tol=1e-10)

    def exact(x, y, z):
        a, b, c = es_velocity(x, y, z, 0.0, nu_l)
        return np.stack([a, b, c, es_pressure(x, y, z, 0.0, nu_l)], axis=-1)
    ev, _ = l2_errors(m.xyz, m.tets, us, exact)
    ei, _ = l2_errors(m.xyz, m.tets, ex, exact)
    return ev, ei


def test_ethier_steinman_velocity_convergence():
    e4, i4 = _es_steady(4, 10.0)
    e8, i8 = _es_steady(8, 10.0)
    assert np.log2(e4 / e8) >= 1.5
    assert e8 <= 2.0 * i8 and e4 <= 2.0 * i4
