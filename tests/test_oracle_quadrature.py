"""Pins of the oracle's quadrature (not gpu).

The exact integral of a barycentric monomial over a tet of volume |T| is
  int l0^a l1^b l2^c l3^d = 3! a! b! c! d! |T| / (a + b + c + d + 3)!
(the classical simplex integration formula).  The bubble moments used by
the closed-form element follow from it with b = 256 l0 l1 l2 l3.
"""
from math import factorial as fac

import numpy as np
import pytest

from oracle.quadrature import tet_rule, gauss_jacobi


def exact_monomial(k):
    return 6.0 * np.prod([fac(int(x)) for x in k]) / fac(int(sum(k)) + 3)


def test_gauss_legendre_matches_numpy():
    for n in (1, 2, 5, 9):
        x, w = gauss_jacobi(n, 0.0, 0.0)
        xr, wr = np.polynomial.legendre.leggauss(n)
        assert np.allclose(np.sort(x), xr, atol=1e-14)
        assert np.allclose(w[np.argsort(x)], wr, atol=1e-14)


@pytest.mark.parametrize("n", [6, 7])
def test_exact_to_degree_2n_minus_1(n):
    lam, w = tet_rule(n)
    assert abs(w.sum() - 1.0 / 6.0) < 1e-15
    deg = 2 * n - 1
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                for d in (deg - a - b - c, max(0, deg - a - b - c - 1)):
                    k = (a, b, c, d)
                    q = 6.0 * np.sum(w * np.prod(lam ** np.array(k), axis=1))
                    ex = exact_monomial(k)
                    assert abs(q - ex) <= 1e-13 * ex, (k, q, ex)


def test_not_exact_beyond_degree():
    lam, w = tet_rule(3)                     # exact to degree 5 only
    k = (0, 0, 0, 8)
    q = 6.0 * np.sum(w * lam[:, 3] ** 8)
    assert abs(q - exact_monomial(k)) > 1e-8


def test_bubble_moments():
    """B = 32/105, B1 = 8/105, C = 8192/51975, grad-bubble energy 4096/945 sum|g|^2 (per |T|)."""
    lam, w = tet_rule(7)
    W = 6.0 * w
    b = 256.0 * np.prod(lam, axis=1)
    assert np.isclose(np.sum(W * b), 32 / 105, rtol=1e-14, atol=0)
    for a in range(4):
        assert np.isclose(np.sum(W * b * lam[:, a]), 8 / 105, rtol=1e-14, atol=0)
    assert np.isclose(np.sum(W * b * b), 8192 / 51975, rtol=1e-14, atol=0)
    # gradient energy on a random tet
    rng = np.random.default_rng(3)
    X = rng.standard_normal((4, 3))
    J = (X[1:] - X[0]).T
    if np.linalg.det(J) < 0:
        X[[2, 3]] = X[[3, 2]]
        J = (X[1:] - X[0]).T
    inv = np.linalg.inv(J)
    g = np.vstack([-inv.sum(axis=0), inv])
    vol = np.linalg.det(J) / 6.0
    db = np.zeros((lam.shape[0], 3))
    for a in range(4):
        prod = 256.0 * np.prod(np.delete(lam, a, axis=1), axis=1)
        db += prod[:, None] * g[a][None, :]
    energy = np.sum(W * vol * np.sum(db * db, axis=1))
    assert np.isclose(energy, 4096 / 945 * vol * np.sum(g * g), rtol=1e-13, atol=0)
    # int grad b = 0 and int b^2 grad b = 0 (b vanishes on the boundary)
    assert np.allclose(np.sum(W[:, None] * db, axis=0), 0, atol=1e-12)
    assert np.allclose(np.sum((W * b * b)[:, None] * db, axis=0), 0, atol=1e-12)
