"""Pins of the oracle's fixed-point (Picard) tangent and iteration (not gpu).

The fixed-point linearisation holds the advecting velocity at the current iterate
(the alternative to the consistent Newton linearisation that the introduction argues
against).  The convective term is bilinear, N(advecting, advected), every other term
of the residual is affine, so:
  * the Picard tangent is the derivative of the residual whose advecting velocity is
    frozen at the state (central differences of an affine function: exact to rounding)
  * Newton minus Picard is the derivative with respect to the advecting velocity alone
  * K_P(U) U = R(U) - R(0) per element (R(0): zero velocity, pressure and fine scales)
  * without flow (v = 0, beta = 0) the two tangents coincide
  * the Picard iteration converges linearly to the Newton solution
"""
import numpy as np
import pytest

from oracle import vms as O
from oracle.element import element_residual_tangent
from workloads import jittered_cube, cavity_mesh, cavity_bc, apply_dirichlet


def _state(mesh, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((mesh.n_nodes, 4))
    up = rng.standard_normal((mesh.n_nodes, 4))
    beta = 0.3 * rng.standard_normal((mesh.n_elems, 3))
    f = rng.standard_normal((mesh.n_nodes, 3))
    return u, up, beta, f


@pytest.fixture(scope="module")
def mesh():
    return jittered_cube(2, seed=11, amp=0.2)


def _perturbed(m, u, beta, e, c, s):
    uu, bb = u.copy(), beta.copy()
    if c < 16:
        uu[m.tets[e, c // 4], c % 4] += s
    else:
        bb[e, c - 16] += s
    return uu, bb


def test_picard_tangent_is_derivative_with_frozen_advection(mesh):
    m = mesh
    u, up, beta, f = _state(m, 3)
    nu, dt = 0.17, 0.04
    sel = [1, 9, 22, 40]
    _, KP = element_residual_tangent(m.xyz, m.tets, u, beta, nu, dt, up, f, picard=True)
    _, KN = element_residual_tangent(m.xyz, m.tets, u, beta, nu, dt, up, f)
    h = 1e-3
    for e in sel:
        for c in range(19):
            def frozen(s):          # advecting velocity held at (u, beta), advected field moved
                uu, bb = _perturbed(m, u, beta, e, c, s)
                return element_residual_tangent(m.xyz, m.tets, uu, bb, nu, dt, up, f, with_tangent=False,
                                                advect=(u, beta))[0][e]

            def advecting(s):      # advected field held, advecting velocity moved
                uu, bb = _perturbed(m, u, beta, e, c, s)
                return element_residual_tangent(m.xyz, m.tets, u, beta, nu, dt, up, f, with_tangent=False,
                                                advect=(uu, bb))[0][e]
            scale = np.max(np.abs(KN[e]))
            fd = (frozen(h) - frozen(-h)) / (2 * h)
            assert np.max(np.abs(fd - KP[e, :, c])) <= 1e-10 * scale, (e, c)
            fd_a = (advecting(h) - advecting(-h)) / (2 * h)
            assert np.max(np.abs(fd_a - (KN[e, :, c] - KP[e, :, c]))) <= 1e-10 * scale, (e, c)


def test_picard_tangent_times_state(mesh):
    m = mesh
    u, up, beta, f = _state(m, 4)
    nu, dt = 0.31, 0.1
    R, KP = element_residual_tangent(m.xyz, m.tets, u, beta, nu, dt, up, f, picard=True)
    R0, _ = element_residual_tangent(m.xyz, m.tets, np.zeros_like(u), np.zeros_like(beta), nu, dt, up, f,
                                     with_tangent=False)
    Ue = np.concatenate([u[m.tets].reshape(-1, 16), beta], axis=1)        # element dof order
    lhs = np.einsum("eij,ej->ei", KP, Ue)
    assert np.max(np.abs(lhs - (R - R0))) <= 1e-12 * np.max(np.abs(R - R0))
    # the Newton tangent counts the convective term twice: K_N U - K_P U = N(U, U)
    _, KN = element_residual_tangent(m.xyz, m.tets, u, beta, nu, dt, up, f)
    conv = np.einsum("eij,ej->ei", KN - KP, Ue)
    Rl, _ = element_residual_tangent(m.xyz, m.tets, u, beta, nu, dt, up, f, with_tangent=False,
                                     advect=(np.zeros_like(u), np.zeros_like(beta)))
    assert np.max(np.abs(conv - (R - Rl))) <= 1e-12 * np.max(np.abs(R - Rl))


def test_picard_equals_newton_without_flow(mesh):
    m = mesh
    rng = np.random.default_rng(5)
    u = np.zeros((m.n_nodes, 4))
    u[:, 3] = rng.standard_normal(m.n_nodes)
    beta = np.zeros((m.n_elems, 3))
    _, KN = element_residual_tangent(m.xyz, m.tets, u, beta, 0.2)
    _, KP = element_residual_tangent(m.xyz, m.tets, u, beta, 0.2, picard=True)
    assert np.array_equal(KN, KP)


def test_picard_iteration_converges_linearly_to_the_newton_solution():
    m = cavity_mesh(3)
    bc = cavity_bc(m)
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    beta = np.zeros((m.n_elems, 3))
    Re = 20.0
    newton = O.Problem(m.xyz, m.tets, bc.dofs, nu=1.0 / Re)
    un, bn, log_n = O.newton_solve(newton, u, beta, tol=1e-11)
    picard = O.Problem(m.xyz, m.tets, bc.dofs, nu=1.0 / Re, picard=True)
    up, bp, log_p = O.newton_solve(picard, u, beta, tol=1e-11, max_newton=80)
    r = np.array(log_p.rnorms)
    assert len(r) > len(log_n.rnorms) + 2                    # linear, not quadratic
    rates = r[3:8] / r[2:7]
    assert np.all(rates < 0.5) and np.ptp(rates) < 0.1, rates
    assert np.linalg.norm(up - un) <= 1e-9 * np.linalg.norm(un)
    assert np.linalg.norm(bp - bn) <= 1e-8 * np.linalg.norm(bn)
