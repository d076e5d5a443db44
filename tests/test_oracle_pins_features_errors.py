"""Pins of two oracle functions against hand-computed values (not gpu).

* oracle.learned_pc.features on a 3-node block matrix written out by hand:
  the diagonal blocks have a Frobenius norm that differs from their largest
  entry, the off-diagonal blocks are not transposes of each other (so row
  and column sums differ), and one dof is Dirichlet.  Every expected number
  below was computed by hand from the matrix in the test.
* oracle.errors.l2_errors against exact integrals over the unit cube: the
  P1 interpolant of a linear field is the field itself and the rule of the
  oracle integrates quadratics exactly, so the error of a linear field
  against another linear field is a closed-form integral, on any mesh of the
  cube (a jittered one is used so that element volumes differ).  A constant
  pressure offset must vanish under the mean removal.
"""
import math

import numpy as np
import scipy.sparse as sp

from oracle import errors
from oracle import learned_pc as lp
from workloads import jittered_cube


def _three_node_matrix():
    # diagonal blocks (row-major 4x4)
    D0 = np.array([[2.0, 1.0, 0.0, 0.0],
                   [0.0, 3.0, 0.0, 0.0],
                   [0.0, 0.0, 4.0, 0.0],
                   [0.0, 0.0, 1.0, -1.0]])
    D1 = np.array([[-5.0, 0.0, 0.0, 2.0],
                   [0.0, 1.0, 0.0, 0.0],
                   [0.0, 0.0, 1.0, 0.0],
                   [2.0, 0.0, 0.0, 0.5]])
    D2 = np.array([[4.0, 0.0, 0.0, 0.0],
                   [0.0, 1.0, 0.0, 0.0],      # dof 4*2+1 is Dirichlet: unit row and column
                   [0.0, 0.0, 2.0, 0.0],
                   [0.0, 0.0, 0.0, -2.0]])
    A01 = np.array([[1.0, -2.0, 0.0, 0.0],
                    [0.0, 0.0, 0.0, 0.0],
                    [0.5, 0.0, 0.0, 0.0],
                    [0.0, 0.0, 0.0, -3.0]])
    A02 = np.array([[0.0, 0.0, 0.0, 1.0],
                    [0.0, 0.0, 0.0, 0.0],
                    [0.0, 0.0, 0.0, 0.0],
                    [0.0, 0.0, 0.0, 0.0]])
    A10 = np.array([[0.0, 6.0, 0.0, 0.0],
                    [0.0, 0.0, 0.0, 0.0],
                    [-1.0, -1.0, 0.0, 0.0],
                    [0.0, 0.0, 0.0, 0.0]])
    A20 = np.array([[0.0, 0.0, 8.0, 0.0],
                    [0.0, 0.0, 0.0, 0.0],
                    [0.0, 0.0, 0.0, 0.0],
                    [0.0, 0.0, 0.0, 4.0]])
    Z = np.zeros((4, 4))
    A = np.block([[D0, A01, A02], [A10, D1, Z], [A20, Z, D2]])
    return sp.csr_matrix(A), (D0, D1, D2)


def test_features_hand_computed():
    A, (D0, D1, D2) = _three_node_matrix()
    x, D = lp.features(A, 3, np.array([9]))
    assert x.shape == (3, 25)
    # Frobenius norms: 4+1+9+16+1+1 = 32;  25+4+1+1+4+0.25 = 35.25;  16+1+4+4 = 25
    fro = [math.sqrt(32.0), math.sqrt(35.25), 5.0]
    for i, Di in enumerate((D0, D1, D2)):
        assert np.allclose(x[i, :16], Di.ravel() / fro[i], rtol=0, atol=1e-15)
        assert abs(x[i, 16] - math.log(fro[i])) < 1e-15
    # row sums of |A_ij[r, :]| over j != i, divided by |D_i[r, r]|:
    #   node 0: rows (3 + 1, 0, 0.5, 3) / (2, 3, 4, 1) = (2, 0, 0.125, 3)
    #   node 1: rows (6, 0, 2, 0) / (5, 1, 1, 0.5)     = (1.2, 0, 2, 0)
    #   node 2: rows (8, 0, 0, 4) / (4, 1, 2, 2)       = (2, 0, 0, 2)
    ratios = [(2.0, 0.0, 0.125, 3.0), (1.2, 0.0, 2.0, 0.0), (2.0, 0.0, 0.0, 2.0)]
    for i, rr in enumerate(ratios):
        assert np.allclose(x[i, 17:21], [math.log(1.0 + v) for v in rr], rtol=0, atol=1e-15), i
    # Dirichlet flags: only dof 1 of node 2
    flags = np.zeros((3, 4))
    flags[2, 1] = 1.0
    assert np.array_equal(x[:, 21:25], flags)
    assert np.array_equal(D, np.stack([D0, D1, D2]))


def test_features_reject_plausible_misreadings():
    """Each misreading of the definition gives numbers that the hand values exclude."""
    A, (D0, _, _) = _three_node_matrix()
    x, _ = lp.features(A, 3, np.array([9]))
    # max-abs normalisation instead of Frobenius
    assert not np.allclose(x[0, :16], D0.ravel() / np.abs(D0).max())
    # column sums instead of row sums: node 0's columns of A10, A20 give (1, 7, 8, 4) / |diag|
    col = [math.log1p(v) for v in (1.0 / 2.0, 7.0 / 3.0, 8.0 / 4.0, 4.0 / 1.0)]
    assert not np.allclose(x[0, 17:21], col)
    # log instead of log1p would be -inf on the zero rows
    assert np.isfinite(x).all()


def _mesh():
    m = jittered_cube(4, seed=3)
    vol6 = np.abs(np.einsum("ei,ei->e", m.xyz[m.tets[:, 1]] - m.xyz[m.tets[:, 0]],
                            np.cross(m.xyz[m.tets[:, 2]] - m.xyz[m.tets[:, 0]],
                                     m.xyz[m.tets[:, 3]] - m.xyz[m.tets[:, 0]])))
    assert vol6.max() > 1.5 * vol6.min()       # element volumes really differ
    return m


def test_l2_velocity_error_of_linear_fields_is_the_exact_integral():
    m = _mesh()
    x, y, z = m.xyz.T
    # exact field f = (1 + x, y, 0); discrete field = f + (0.1 z, 0, 0.2 x)
    u = np.stack([1.0 + x + 0.1 * z, y, 0.2 * x, np.zeros_like(x)], axis=1)

    def exact(X, Y, Z):
        return np.stack([1.0 + X, Y, 0.0 * X, X], axis=-1)

    ev, _ = errors.l2_errors(m.xyz, m.tets, u, exact)
    # int (0.1 z)^2 + (0.2 x)^2 = 0.01/3 + 0.04/3;  int (1 + x)^2 + y^2 = 7/3 + 1/3
    assert abs(ev - math.sqrt((0.05 / 3.0) / (8.0 / 3.0))) < 1e-13


def test_l2_pressure_error_is_mean_free():
    m = _mesh()
    x, y, z = m.xyz.T
    # exact p = x; discrete p = x + 7 + 0.5 (y - 1/2): the constant 7 must not count
    u = np.zeros((m.n_nodes, 4))
    u[:, 0] = 1.0
    u[:, 3] = x + 7.0 + 0.5 * (y - 0.5)

    def exact(X, Y, Z):
        return np.stack([1.0 + 0.0 * X, 0.0 * X, 0.0 * X, X], axis=-1)

    ev, ep = errors.l2_errors(m.xyz, m.tets, u, exact)
    assert ev < 1e-14
    # int (0.5 (y - 1/2))^2 = 1/48;  int (x - 1/2)^2 = 1/12
    assert abs(ep - 0.5) < 1e-13


def test_l2_errors_weight_elements_by_volume():
    """A uniform weight per element (|T| left out) gives another value on this mesh."""
    m = _mesh()
    x, y, z = m.xyz.T
    u = np.stack([1.0 + x + 0.1 * z, y, 0.2 * x, np.zeros_like(x)], axis=1)

    def exact(X, Y, Z):
        return np.stack([1.0 + X, Y, 0.0 * X, X], axis=-1)

    ev, _ = errors.l2_errors(m.xyz, m.tets, u, exact)
    from oracle.quadrature import tet_rule
    lam, w = tet_rule(5)
    X = m.xyz[m.tets]
    pts = np.einsum("qa,eai->eqi", lam, X)
    uh = np.einsum("qa,eac->eqc", lam, u[m.tets])
    ex = exact(pts[..., 0], pts[..., 1], pts[..., 2])
    unweighted = math.sqrt(np.sum(w * np.sum((uh[..., :3] - ex[..., :3]) ** 2, axis=-1))
                           / np.sum(w * np.sum(ex[..., :3] ** 2, axis=-1)))
    assert abs(unweighted - ev) > 1e-4 * ev
