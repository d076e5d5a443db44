"""Pins of the oracle's GMRES with deflated restarting (oracle/gmres_dr.py), not gpu.

* k = 0 is plain restarted GMRES: the same steps, cycles and iterate as the oracle's textbook
  GMRES(m) (Givens rotations, modified Gram-Schmidt) on a condensed backward-facing-step system.
* A diagonal matrix with four isolated small eigenvalues (1e-3 .. 1e-2) under a spectrum in
  [1, 10]: the kept harmonic Ritz values are those eigenvalues (harmonic Ritz values converge
  to the eigenvalues nearest zero), and removing them cuts the steps of GMRES(20) tenfold.
* A complex pair 0.01 (1 +- i) next to a real 0.003: with k = 2 the pair is kept whole (three
  values), each to its closed form.
* The deflated solve of the condensed system meets rtol and agrees with the direct solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import vms as O
from oracle.gmres_dr import gmres_dr
from workloads import backward_facing_step, bfs_bc, apply_dirichlet


@pytest.fixture(scope="module")
def bfs_system():
    m = backward_facing_step(1, 2, 1)
    bc = bfs_bc(m)
    u = np.zeros((m.n_nodes, 4))
    apply_dirichlet(u, bc)
    prob = O.Problem(m.xyz, m.tets, bc.dofs, 1.0 / 50.0)
    A, b, _, _ = O.condensed_system(prob, u, np.zeros((m.n_elems, 3)))
    return A, b, O.block_jacobi_inverse(A, m.n_nodes)


def test_no_deflation_is_textbook_restarted_gmres(bfs_system):
    A, b, Mb = bfs_system
    g = O.gmres(A, b, restart=30, rtol=1e-10, max_iters=20000, Minv_blocks=Mb)
    r = gmres_dr(A, b, restart=30, k=0, rtol=1e-10, max_iters=20000, Minv_blocks=Mb)
    assert g.converged and r.converged
    assert (r.iters, r.restarts) == (g.iters, g.restarts)
    assert np.linalg.norm(r.x - g.x) <= 1e-8 * np.linalg.norm(g.x)


def test_deflated_solve_matches_the_direct_solution(bfs_system):
    A, b, Mb = bfs_system
    r = gmres_dr(A, b, restart=30, k=10, rtol=1e-10, max_iters=20000, Minv_blocks=Mb)
    g = gmres_dr(A, b, restart=30, k=0, rtol=1e-10, max_iters=20000, Minv_blocks=Mb)
    xd = O.solve_direct(A, b)
    assert r.converged and np.linalg.norm(b - A @ r.x) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(r.x - xd) <= 1e-7 * np.linalg.norm(xd)
    assert r.iters * 4 < g.iters


def test_kept_values_are_the_isolated_eigenvalues():
    rng = np.random.default_rng(3)
    n = 1000
    small = np.array([1e-3, 2e-3, 5e-3, 1e-2])
    lam = np.concatenate([small, 1.0 + 9.0 * rng.random(n - 4)])
    A = sp.diags(lam).tocsr()
    b = rng.standard_normal(n)
    plain = gmres_dr(A, b, restart=20, k=0, rtol=1e-10, max_iters=20000)
    dr = gmres_dr(A, b, restart=20, k=4, rtol=1e-10, max_iters=20000)
    assert plain.converged and dr.converged
    th = np.sort(dr.theta.real)
    assert np.all(dr.theta.imag == 0) and th.size == 4
    assert np.abs(th - small).max() <= 1e-7 * small.min()
    assert dr.iters * 10 <= plain.iters
    assert np.linalg.norm(dr.x - b / lam) <= 1e-8 * np.linalg.norm(b / lam)


def test_a_complex_pair_is_kept_whole():
    rng = np.random.default_rng(4)
    n = 400
    blocks = [np.array([[0.01, 0.01], [-0.01, 0.01]]), np.array([[0.003]])]
    A = sp.block_diag(blocks + [sp.diags(1.0 + rng.random(n - 3))]).tocsr()
    b = rng.standard_normal(n)
    r = gmres_dr(A, b, restart=20, k=2, rtol=1e-10, max_iters=20000)
    assert r.converged and r.theta.size == 3
    want = np.array([0.003, 0.01 + 0.01j, 0.01 - 0.01j])
    got = r.theta[np.argsort(np.abs(r.theta) + 1e-9 * np.sign(-r.theta.imag))]
    assert np.abs(got - want).max() <= 1e-9
