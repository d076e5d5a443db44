"""Jet from an orifice on the GPU (Section 5 transient jet case), through the C ABI.

The paper gives the case in a figure that is not available; the geometry here is a reading
of its caption: an orifice of diameter 1 in a no-slip wall (x = 0) with a parabolic inflow of
peak 1 along x, every other face traction-free (no pressure pin), Re 1000, backward Euler
with dt 0.01, impulsive start from rest.

* Two time steps on the 8^3-cell box (3,072 tets): the GPU Newton-Schur iterates against the
  oracle's own time stepping, FP64 to 1e-9 and mixed precision to 1e-5.
* The full-size case (32^3 cells x 6 = 196,608 tets), a few mixed-precision steps, checked on
  sampled outputs the oracle computes one by one: the assembled FP64 residual at sampled free
  nodes (wall-free interior and the traction-free faces) and the fine-scale residual of sampled
  elements in the final state.
"""
import functools

import numpy as np
import pytest
import torch

from oracle import vms as O
from oracle.element import element_residual_tangent
from workloads import jet_box, jet_bc, apply_dirichlet, build_workload
from tests.gpu_common import DEV, to_dev, make_context, rel_fro

pytestmark = pytest.mark.gpu


def _march(B, ctx, m, bc, u, beta, Re, dt, steps, lin, tol):
    """Backward Euler on the GPU; the wall values do not change in time.  Returns the
    per-step Newton results and the state before the last step."""
    from paper_0809_4802_amd import driver
    dofs = to_dev(bc.dofs.astype(np.int64))
    vals = to_dev(bc.values)
    u_prev = torch.empty_like(u)
    out = []
    for _ in range(steps):
        u_prev.copy_(u)
        driver.set_dirichlet(u, dofs, vals)
        out.append(driver.newton_solve(ctx, u, beta, Re, dt, u_prev, None, tol=tol, lin=lin))
    return out, u_prev


@functools.lru_cache(maxsize=None)
def _oracle_march(c, Re, dt, steps):
    """The oracle's backward Euler on jet_box(c) (computed once for both precisions)."""
    m = jet_box(c)
    bc = jet_bc(m)
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    beta = np.zeros((m.n_elems, 3))
    for _ in range(steps):
        up = u.copy()
        prob = O.Problem(m.xyz, m.tets, bc.dofs, nu=1.0 / Re, dt=dt, u_prev=up)
        u, beta, _ = O.newton_solve(prob, u, beta, tol=1e-12)
    return u, beta


@pytest.mark.parametrize("precision", [0, 1])
def test_jet_backward_euler_matches_oracle(vms_lib, precision):
    B = vms_lib
    m = jet_box(2)
    bc = jet_bc(m)
    assert not np.any(bc.dofs % 4 == 3)
    Re, dt, steps = 1000.0, 0.01, 2
    u0 = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u0, bc)
    ctx = make_context(B, m, bc.dofs, precision)
    ud = to_dev(u0)
    bd = torch.zeros((m.n_elems, 3), dtype=torch.float64, device=DEV)
    fp64 = precision == B.VMS_FP64
    tol = 1e-11 if fp64 else 1e-8
    res, _ = _march(B, ctx, m, bc, ud, bd, Re, dt, steps, B.solve_opts(rtol=tol / 10, max_iters=40000), tol)
    assert all(r.converged for r in res)
    u, beta = _oracle_march(2, Re, dt, steps)
    print(f"jet 8^3 {'fp64' if fp64 else 'mixed'}: Newton steps {[len(r.rnorms) - 1 for r in res]}, "
          f"GMRES iterations {[sum(d['iters'] for d in r.lin) for r in res]}")
    assert rel_fro(ud.cpu().numpy(), u) <= (1e-9 if fp64 else 1e-5)
    assert rel_fro(bd.cpu().numpy(), beta) <= (1e-7 if fp64 else 1e-4)


def _patch_residuals(m, u, beta, nu, dt, u_prev, nodes, elems):
    """Oracle FP64 residuals: assembled [R_c; R_p] at the given nodes (from every element
    touching them) and the fine-scale R_f of the given elements."""
    patch = np.nonzero(np.isin(m.tets, nodes).any(axis=1))[0]
    R, _ = element_residual_tangent(m.xyz, m.tets[patch], u, beta[patch], nu, dt, u_prev, None,
                                    with_tangent=False)
    Rn = np.zeros((nodes.size, 4))
    where = {int(v): i for i, v in enumerate(nodes)}
    for k, e in enumerate(patch):
        for a in range(4):
            i = where.get(int(m.tets[e, a]))
            if i is not None:
                Rn[i] += R[k, 4 * a:4 * a + 4]
    Rf, _ = element_residual_tangent(m.xyz, m.tets[elems], u, beta[elems], nu, dt, u_prev, None,
                                     with_tangent=False)
    return Rn, Rf[:, 16:19]


def test_jet8_transient_full_size(vms_lib):
    B = vms_lib
    cfg, m, u0, beta0, bc = build_workload("jet8")
    assert m.n_elems == 196_608 and cfg.re == 1000.0 and cfg.dt == 0.01
    steps = 3
    ctx = make_context(B, m, bc.dofs, B.VMS_MIXED)
    ud = to_dev(u0)
    bd = to_dev(beta0)
    res, u_prev = _march(B, ctx, m, bc, ud, bd, cfg.re, cfg.dt, steps,
                         B.solve_opts(rtol=1e-9, max_iters=40000), cfg.newton_tol)
    assert all(r.converged for r in res)
    u, beta, up = ud.cpu().numpy(), bd.cpu().numpy(), u_prev.cpu().numpy()
    print(f"jet8: Newton steps {[len(r.rnorms) - 1 for r in res]}, "
          f"GMRES iterations {[sum(d['iters'] for d in r.lin) for r in res]}, "
          f"seconds per step {[round(r.seconds, 3) for r in res]}, max u_x {u[:, 0].max():.3f}")
    assert np.all(np.isfinite(u)) and np.all(np.isfinite(beta))
    # the fluid next to the orifice centre moves into the box along +x
    axis = int(np.argmin(np.sum((m.xyz - np.array([0.125, 0.0, 0.0])) ** 2, axis=1)))
    assert u[axis, 0] > 0.1
    # oracle residual of the final state at sampled free nodes (some on the traction-free
    # faces) and sampled elements
    rng = np.random.default_rng(11)
    free = np.setdiff1d(np.arange(m.n_nodes), bc.dofs // 4)
    x = m.xyz[free]
    on_face = free[(np.abs(np.abs(x[:, 1]) - 2.0) < 1e-12) | (np.abs(np.abs(x[:, 2]) - 2.0) < 1e-12)
                   | (np.abs(x[:, 0] - 4.0) < 1e-12)]
    nodes = np.unique(np.concatenate([rng.choice(free, size=48, replace=False),
                                      rng.choice(on_face, size=16, replace=False)]))
    elems = np.sort(rng.choice(m.n_elems, size=256, replace=False))
    Rn, Rf = _patch_residuals(m, u, beta, 1.0 / cfg.re, cfg.dt, up, nodes, elems)
    r0 = res[-1].rnorms[0]
    assert np.abs(Rn).max() <= 1.01 * cfg.newton_tol * r0, (np.abs(Rn).max(), r0)
    assert np.abs(Rf).max() <= 1.01 * cfg.newton_tol * r0, (np.abs(Rf).max(), r0)
