"""Seeded synthetic inputs shared by the product path, the oracle and the tests.

This package generates meshes, boundary data and manufactured fields.  It
holds none of the variational multiscale arithmetic: no residual, tangent,
condensation or solver code lives here.
"""
from .mesh import (Mesh, kuhn_box, jittered_cube, cavity_mesh, backward_facing_step, jet_box,
                   boundary_nodes, tet_volumes6, count_edges, jitter_interior)
from .bc import (DirichletData, cavity_bc, ethier_steinman_bc, bfs_bc, jet_bc, apply_dirichlet)
from .ethier_steinman import es_velocity, es_pressure, ES_A, ES_D
from .configs import CONFIGS, WorkloadConfig, build_workload

__all__ = [
    "Mesh", "kuhn_box", "jittered_cube", "cavity_mesh", "backward_facing_step", "jet_box",
    "boundary_nodes", "tet_volumes6", "count_edges", "jitter_interior",
    "DirichletData", "cavity_bc", "ethier_steinman_bc", "bfs_bc", "jet_bc", "apply_dirichlet",
    "es_velocity", "es_pressure", "ES_A", "ES_D",
    "CONFIGS", "WorkloadConfig", "build_workload",
]
