"""Quadrature on the tetrahedron for the oracle (test infrastructure).

Conical-product (Stroud) rule: the unit cube (s, t, r) is collapsed onto the
reference tet {x, y, z >= 0, x + y + z <= 1} by
    x = s,  y = t (1 - s),  z = r (1 - s)(1 - t),
whose Jacobian is (1 - s)^2 (1 - t).  Gauss-Jacobi rules with weights
(1 - s)^2 and (1 - t) and a Gauss-Legendre rule in r, n points each, are
exact for polynomials of total degree 2n - 1 on the tet.  The 1-D rules are
built by the Golub-Welsch method: the nodes are the eigenvalues of the
symmetric tridiagonal Jacobi matrix of the orthogonal polynomials, the
weights come from the first components of its eigenvectors.

The paper does not name a quadrature rule.  Every integrand of the element
residual and tangent is a polynomial of degree at most 11 in the barycentric
coordinates on an affine tet, so the oracle integrates exactly (n = 7 is
exact to degree 13).
"""
from __future__ import annotations

from functools import lru_cache
from math import gamma

import numpy as np


def gauss_jacobi(n: int, alpha: float, beta: float):
    """n-point Gauss-Jacobi rule on [-1, 1] for weight (1-x)^alpha (1+x)^beta."""
    k = np.arange(n, dtype=np.float64)
    ab = alpha + beta
    diag = np.empty(n)
    with np.errstate(divide="ignore", invalid="ignore"):
        diag[:] = (beta ** 2 - alpha ** 2) / ((2 * k + ab) * (2 * k + ab + 2))
    if abs(ab) < 1e-300:
        diag[0] = (beta - alpha) / (ab + 2)
    kk = np.arange(1, n, dtype=np.float64)
    off = np.sqrt(4 * kk * (kk + alpha) * (kk + beta) * (kk + ab)
                  / ((2 * kk + ab) ** 2 * (2 * kk + ab + 1) * (2 * kk + ab - 1)))
    jac = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    x, vec = np.linalg.eigh(jac)
    mu0 = 2.0 ** (ab + 1) * gamma(alpha + 1) * gamma(beta + 1) / gamma(ab + 2)
    w = mu0 * vec[0, :] ** 2
    return x, w


def gauss_jacobi01(n: int, alpha: float):
    """Rule on [0, 1] for the weight (1 - s)^alpha."""
    x, w = gauss_jacobi(n, alpha, 0.0)
    return 0.5 * (x + 1.0), w * 0.5 ** (alpha + 1.0)


@lru_cache(maxsize=None)
def tet_rule(n: int = 7):
    """(lam [nq, 4], w [nq]) on the reference tet; sum(w) = 1/6.

    lam are barycentric coordinates (lam0 = 1 - x - y - z, lam1 = x,
    lam2 = y, lam3 = z).  Multiply w by 6|T| for a physical tet of volume |T|.
    """
    s, ws = gauss_jacobi01(n, 2.0)
    t, wt = gauss_jacobi01(n, 1.0)
    r, wr = gauss_jacobi01(n, 0.0)
    S, T, R = np.meshgrid(s, t, r, indexing="ij")
    W = ws[:, None, None] * wt[None, :, None] * wr[None, None, :]
    x = S
    y = T * (1 - S)
    z = R * (1 - S) * (1 - T)
    lam = np.stack([1 - x - y - z, x, y, z], axis=-1).reshape(-1, 4)
    w = W.reshape(-1)
    lam.setflags(write=False)
    w.setflags(write=False)
    return lam, w
