"""Ethier-Steinman three-dimensional Beltrami flow (manufactured solution).

Exact unsteady solution of the incompressible Navier-Stokes equations
  du/dt + (u.grad)u - nu_L lap(u) + grad(p) = 0,  div(u) = 0
with a = pi/4, d = pi/2 and decay E(t) = exp(-nu_L d^2 t).  The paper's
momentum equation carries the viscous coefficient 2 nu on the Laplacian
(Section 2, balance of linear momentum), so a run at viscosity nu uses
nu_L = 2 nu.  p is the kinematic pressure.
"""
from __future__ import annotations

import numpy as np

ES_A = np.pi / 4.0
ES_D = np.pi / 2.0


def es_velocity(x, y, z, t, nu_l, a=ES_A, d=ES_D):
    """Velocity (u, v, w), each shaped like x."""
    e = np.exp(-nu_l * d * d * t)
    u = -a * (np.exp(a * x) * np.sin(a * y + d * z) + np.exp(a * z) * np.cos(a * x + d * y)) * e
    v = -a * (np.exp(a * y) * np.sin(a * z + d * x) + np.exp(a * x) * np.cos(a * y + d * z)) * e
    w = -a * (np.exp(a * z) * np.sin(a * x + d * y) + np.exp(a * y) * np.cos(a * z + d * x)) * e
    return u, v, w


def es_pressure(x, y, z, t, nu_l, a=ES_A, d=ES_D):
    """Kinematic pressure, written out term by term (it equals -|u|^2 / 2)."""
    e2 = np.exp(-2.0 * nu_l * d * d * t)
    return -0.5 * a * a * e2 * (
        np.exp(2 * a * x) + np.exp(2 * a * y) + np.exp(2 * a * z)
        + 2 * np.sin(a * x + d * y) * np.cos(a * z + d * x) * np.exp(a * (y + z))
        + 2 * np.sin(a * y + d * z) * np.cos(a * x + d * y) * np.exp(a * (z + x))
        + 2 * np.sin(a * z + d * x) * np.cos(a * y + d * z) * np.exp(a * (x + y)))


def es_nodal(xyz, t, nu_l):
    """Nodal interpolant [n_nodes, 4] = (u, v, w, p) of the exact field at time t."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    u, v, w = es_velocity(x, y, z, t, nu_l)
    p = es_pressure(x, y, z, t, nu_l)
    return np.stack([u, v, w, p], axis=1)
