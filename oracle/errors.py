"""ORACLE (test infrastructure): L2 errors against a closed-form field.

The discrete velocity compared is the coarse (nodal P1) velocity; the
pressure is compared after removing its mean from both fields.  Integrals
use the conical-product rule with n points per direction on every tet.
"""
from __future__ import annotations

import numpy as np

from .quadrature import tet_rule


def l2_errors(xyz, tets, u, exact_fn, n_quad=5):
    """Relative L2 errors (velocity, mean-free pressure) of the P1 field u
    [n_nodes, 4] against exact_fn(x, y, z) -> [..., 4]."""
    lam, w = tet_rule(n_quad)
    X = xyz[tets]                                        # [E, 4, 3]
    e1, e2, e3 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]
    det = np.einsum("ei,ei->e", e1, np.cross(e2, e3))    # 6 |T|
    pts = np.einsum("qa,eai->eqi", lam, X)               # [E, Q, 3]
    uh = np.einsum("qa,eac->eqc", lam, u[tets])          # [E, Q, 4]
    ex = exact_fn(pts[..., 0], pts[..., 1], pts[..., 2])
    wq = w[None, :] * det[:, None]
    vol = wq.sum()
    ev = np.sum(wq * np.sum((uh[..., :3] - ex[..., :3]) ** 2, axis=-1))
    nv = np.sum(wq * np.sum(ex[..., :3] ** 2, axis=-1))
    ph = uh[..., 3] - np.sum(wq * uh[..., 3]) / vol
    pe = ex[..., 3] - np.sum(wq * ex[..., 3]) / vol
    ep = np.sum(wq * (ph - pe) ** 2)
    npn = np.sum(wq * pe ** 2)
    return float(np.sqrt(ev / nv)), float(np.sqrt(ep / npn))
