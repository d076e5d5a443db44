"""Dirichlet data for the four workload families.

A Dirichlet dof is 4*node + c with c = 0, 1, 2 the velocity components and
c = 3 the pressure.  The solvers work on Newton increments, so the
prescribed values are written into the state before each solve and the
increment at a Dirichlet dof is zero.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .mesh import Mesh, boundary_nodes
from .ethier_steinman import es_nodal


@dataclass
class DirichletData:
    dofs: np.ndarray        # int32 [n_dirichlet], sorted, unique
    values: np.ndarray      # float64 [n_dirichlet]

    @property
    def n(self) -> int:
        return int(self.dofs.size)


def _pack(node_ids, comps, values):
    dofs = (4 * np.asarray(node_ids, dtype=np.int64) + np.asarray(comps, dtype=np.int64))
    order = np.argsort(dofs, kind="stable")
    dofs = dofs[order]
    vals = np.asarray(values, dtype=np.float64)[order]
    if np.unique(dofs).size != dofs.size:
        raise ValueError("duplicate Dirichlet dof")
    return DirichletData(dofs=dofs.astype(np.int32), values=vals)


def _nearest_node(xyz, point):
    return int(np.argmin(np.sum((xyz - np.asarray(point)) ** 2, axis=1)))


def cavity_bc(mesh: Mesh, lid=(1.0, 0.0, 0.0)) -> DirichletData:
    """No-slip walls, lid velocity on z = 1 (open face only: walls win on
    lid edges), pressure pinned to 0 at the node nearest the centre."""
    x = mesh.xyz
    bnd = np.nonzero(boundary_nodes(mesh.tets, mesh.n_nodes))[0]
    eps = 1e-12
    on_lid = ((np.abs(x[bnd, 2] - 1.0) < eps) & (x[bnd, 0] > eps) & (x[bnd, 0] < 1 - eps)
              & (x[bnd, 1] > eps) & (x[bnd, 1] < 1 - eps))
    vel = np.zeros((bnd.size, 3))
    vel[on_lid] = np.asarray(lid, dtype=np.float64)
    nodes = np.repeat(bnd, 3)
    comps = np.tile(np.arange(3), bnd.size)
    pin = _nearest_node(x, (0.5, 0.5, 0.5))
    return _pack(np.concatenate([nodes, [pin]]), np.concatenate([comps, [3]]),
                 np.concatenate([vel.ravel(), [0.0]]))


def ethier_steinman_bc(mesh: Mesh, t: float, nu_l: float) -> DirichletData:
    """Exact velocity at time t on every boundary node; pressure pinned to the
    exact value at the node nearest the centre."""
    bnd = np.nonzero(boundary_nodes(mesh.tets, mesh.n_nodes))[0]
    ex = es_nodal(mesh.xyz, t, nu_l)
    pin = _nearest_node(mesh.xyz, (0.5, 0.5, 0.5))
    nodes = np.concatenate([np.repeat(bnd, 3), [pin]])
    comps = np.concatenate([np.tile(np.arange(3), bnd.size), [3]])
    vals = np.concatenate([ex[bnd, :3].ravel(), [ex[pin, 3]]])
    return _pack(nodes, comps, vals)


def bfs_bc(mesh: Mesh, u_max: float = 1.0) -> DirichletData:
    """Backward-facing step: parabolic inflow at x = -5, no-slip on every wall
    (including the step face and top), traction-free outlet at x = 30 (no
    Dirichlet dof on the open outlet face, no pressure pin)."""
    x = mesh.xyz
    bnd = np.nonzero(boundary_nodes(mesh.tets, mesh.n_nodes))[0]
    xb = x[bnd]
    eps = 1e-9
    outlet_open = ((np.abs(xb[:, 0] - 30.0) < eps) & (xb[:, 1] > eps) & (xb[:, 1] < 2 - eps)
                   & (xb[:, 2] > eps) & (xb[:, 2] < 4 - eps))
    nodes = bnd[~outlet_open]
    xn = x[nodes]
    inlet = np.abs(xn[:, 0] + 5.0) < eps
    vel = np.zeros((nodes.size, 3))
    y, z = xn[inlet, 1], xn[inlet, 2]
    vel[inlet, 0] = u_max * 4.0 * (y - 1.0) * (2.0 - y) * z * (4.0 - z) / 4.0
    return _pack(np.repeat(nodes, 3), np.tile(np.arange(3), nodes.size), vel.ravel())


def jet_bc(mesh: Mesh, radius: float = 0.5, u_max: float = 1.0) -> DirichletData:
    """Jet from an orifice: every node of the wall x = 0 has its velocity prescribed, the
    paraboloid u_x = u_max (1 - r^2 / radius^2) inside the orifice (r = distance from the
    orifice centre, the origin; zero on its rim) and no slip elsewhere.  The other five
    faces are traction-free: no Dirichlet dof there and no pressure pin."""
    x = mesh.xyz
    nodes = np.nonzero(np.abs(x[:, 0]) < 1e-9)[0]
    r2 = x[nodes, 1] ** 2 + x[nodes, 2] ** 2
    vel = np.zeros((nodes.size, 3))
    vel[:, 0] = u_max * np.maximum(0.0, 1.0 - r2 / radius ** 2)
    return _pack(np.repeat(nodes, 3), np.tile(np.arange(3), nodes.size), vel.ravel())


def apply_dirichlet(u: np.ndarray, bc: DirichletData) -> np.ndarray:
    """Write the prescribed values into a state u [n_nodes, 4] (in place)."""
    flat = u.reshape(-1)
    flat[bc.dofs] = bc.values
    return u
