"""The six synthetic workloads (meshes, physics and tolerances).

  cavity4   steady lid-driven cavity, 4^3 cells x 6 tets, Re 1, FP64,
            Newton to 1e-10, linear rtol 1e-12 (small parity case)
  cavity32  steady lid-driven cavity, 32^3 x 6 tets, Re 100, Newton to 1e-8,
            GMRES(50) + block-Jacobi; FP64 vs mixed precision
  es64      jittered unit cube 64^3 x 6 tets (seed 0, +-0.2h), Ethier-Steinman
            Beltrami flow, Re 1000, backward Euler dt 0.01, 10 steps, mixed
  bfs8      backward-facing step, (8,10,10) cells per unit length (1,248,000
            tets), steady Re 400..800 continuation, mixed; training data for
            the learned preconditioner
  bfs16     backward-facing step, (16,10,10) (2,496,000 tets), Re 800,
            dt 0.05, 50 steps, learned vs plain block-Jacobi
  jet8      jet from an orifice (diameter 1) in a no-slip wall, box 4^3 with 8
            cells per unit length (32^3 x 6 = 196,608 tets), traction-free
            elsewhere, Re 1000, backward Euler dt 0.01 from rest, mixed
Velocity and length scales are 1 everywhere, so nu = 1 / Re.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .mesh import cavity_mesh, jittered_cube, backward_facing_step, jet_box
from .bc import cavity_bc, ethier_steinman_bc, bfs_bc, jet_bc, apply_dirichlet
from .ethier_steinman import es_nodal


@dataclass(frozen=True)
class WorkloadConfig:
    name: str
    family: str                  # "cavity" | "es" | "bfs" | "jet"
    mesh_args: tuple
    re: float
    dt: float                    # <= 0: steady
    steps: int                   # time steps (1 for steady)
    newton_tol: float
    linear_rtol: float
    precision: str               # "fp64" | "mixed"
    re_sweep: tuple = field(default=())


CONFIGS = {
    "cavity4": WorkloadConfig("cavity4", "cavity", (4,), 1.0, 0.0, 1, 1e-10, 1e-12, "fp64"),
    "cavity32": WorkloadConfig("cavity32", "cavity", (32,), 100.0, 0.0, 1, 1e-8, 1e-8, "mixed"),
    "es64": WorkloadConfig("es64", "es", (64, 0), 1000.0, 0.01, 10, 1e-8, 1e-8, "mixed"),
    "bfs8": WorkloadConfig("bfs8", "bfs", (8, 10, 10), 800.0, 0.0, 1, 1e-8, 1e-8, "mixed",
                           re_sweep=(400.0, 500.0, 600.0, 700.0, 800.0)),
    "bfs16": WorkloadConfig("bfs16", "bfs", (16, 10, 10), 800.0, 0.05, 50, 1e-8, 1e-8, "mixed"),
    "jet8": WorkloadConfig("jet8", "jet", (8,), 1000.0, 0.01, 100, 1e-8, 1e-8, "mixed"),
}


def make_mesh(cfg: WorkloadConfig):
    if cfg.family == "cavity":
        return cavity_mesh(*cfg.mesh_args)
    if cfg.family == "es":
        n, seed = cfg.mesh_args
        return jittered_cube(n, seed=seed)
    if cfg.family == "bfs":
        return backward_facing_step(*cfg.mesh_args)
    if cfg.family == "jet":
        return jet_box(*cfg.mesh_args)
    raise ValueError(cfg.family)


def initial_state(cfg: WorkloadConfig, mesh, t: float = 0.0):
    """(u [n_nodes, 4], beta [n_elems, 3], bc) at time t, BCs written into u."""
    nu_l = 2.0 / cfg.re
    if cfg.family == "cavity":
        bc = cavity_bc(mesh)
        u = np.zeros((mesh.n_nodes, 4))
    elif cfg.family == "es":
        bc = ethier_steinman_bc(mesh, t, nu_l)
        u = es_nodal(mesh.xyz, t, nu_l)
    elif cfg.family == "jet":
        bc = jet_bc(mesh)
        u = np.zeros((mesh.n_nodes, 4))
    else:
        bc = bfs_bc(mesh)
        u = np.zeros((mesh.n_nodes, 4))
    apply_dirichlet(u, bc)
    beta = np.zeros((mesh.n_elems, 3))
    return u, beta, bc


def build_workload(name: str):
    cfg = CONFIGS[name]
    mesh = make_mesh(cfg)
    u, beta, bc = initial_state(cfg, mesh)
    return cfg, mesh, u, beta, bc
