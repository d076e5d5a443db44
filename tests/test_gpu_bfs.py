"""Backward-facing step on the GPU (open outlet, no pressure pin), through the C ABI.

The outlet is traction-free, so no pressure dof is prescribed and the constant-pressure
coarse correction must stay off.  A coarse channel with (1, 2, 1) cells per unit length,
3,120 tets, is small enough for the oracle's direct solves; two cells across the inlet give
it an interior inlet row, so the inflow (and the solution) is not zero.
"""
import numpy as np
import pytest
import torch

from oracle import vms as O
from workloads import backward_facing_step, bfs_bc, apply_dirichlet
from tests.gpu_common import DEV, to_dev, make_context, rel_fro

pytestmark = pytest.mark.gpu


def _bfs():
    m = backward_facing_step(1, 2, 1)
    bc = bfs_bc(m)
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    assert not np.any(bc.dofs % 4 == 3)          # no pressure dof is prescribed
    assert np.isclose(bc.values.max(), 1.0)       # inflow peak at the inlet row y = 1.5, z = 2
    return m, bc, u


@pytest.mark.parametrize("precision", [0, 1])
def test_bfs_steady_newton_matches_oracle(vms_lib, precision):
    from paper_0809_4802_amd import driver
    B = vms_lib
    m, bc, u = _bfs()
    Re = 50.0
    ctx = make_context(B, m, bc.dofs, precision)
    ud = to_dev(u)
    bd = torch.zeros((m.n_elems, 3), dtype=torch.float64, device=DEV)
    tol = 1e-10 if precision == B.VMS_FP64 else 1e-8
    res = driver.newton_solve(ctx, ud, bd, Re, tol=tol, lin=B.solve_opts(rtol=tol / 10, max_iters=40000))
    assert res.converged
    prob = O.Problem(m.xyz, m.tets, bc.dofs, nu=1.0 / Re)
    rn = O.residual_norm_at(prob, ud.cpu().numpy(), bd.cpu().numpy())
    assert rn <= 1.01 * tol * res.rnorms[0]
    us, _, _ = O.newton_solve(prob, u, np.zeros((m.n_elems, 3)), tol=1e-12)
    free = np.setdiff1d(np.arange(m.n_nodes), bc.dofs // 4)
    assert np.abs(us[free, 0]).max() > 0.1        # a flow through the free nodes, not the zero state
    assert rel_fro(ud.cpu().numpy(), us) <= (1e-8 if precision == B.VMS_FP64 else 1e-5)
