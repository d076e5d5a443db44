"""Input generators and the manufactured solution (not gpu).

  * Kuhn split counts have closed forms: 6 n^3 tets, (n+1)^3 nodes and
    3n(n+1)^2 + 3n^2(n+1) + n^3 edges; nonzero 4x4 blocks = nodes + 2 edges
  * the paper's Table 1 (fine DOF = 3 per element: one bubble with three
    components per tet; total = coarse + fine) is read from a cited fixture
  * the Ethier-Steinman field satisfies the Navier-Stokes equations with
    Laplacian coefficient nu_L (finite-difference substitution)
"""
import os

import numpy as np
import pytest

from workloads import (cavity_mesh, jittered_cube, backward_facing_step, jet_box, boundary_nodes,
                       count_edges, tet_volumes6, cavity_bc, bfs_bc, jet_bc, ethier_steinman_bc,
                       es_velocity, es_pressure, CONFIGS)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", [1, 2, 4, 7])
def test_kuhn_counts(n):
    m = cavity_mesh(n)
    assert m.n_elems == 6 * n ** 3
    assert m.n_nodes == (n + 1) ** 3
    edges = 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3
    assert count_edges(m.tets, m.n_nodes) == edges
    assert np.all(tet_volumes6(m.xyz, m.tets) > 0)
    assert np.isclose(tet_volumes6(m.xyz, m.tets).sum() / 6, 1.0)


def test_cavity32_sizes():
    m = cavity_mesh(32)
    assert (m.n_elems, m.n_nodes) == (196608, 35937)
    assert m.n_nodes + 2 * count_edges(m.tets, m.n_nodes) == 513313


def test_bfs_sizes_and_volume():
    m = backward_facing_step(8, 10, 10)
    assert (m.n_elems, m.n_nodes) == (1248000, 225541)
    assert np.isclose(tet_volumes6(m.xyz, m.tets).sum() / 6, 5 * 1 * 4 + 30 * 2 * 4)
    bc = bfs_bc(m)
    assert np.isclose(bc.values.max(), 1.0)
    assert not np.any(bc.dofs % 4 == 3)          # no pressure pin: open outlet


def test_jet_sizes_and_orifice():
    m = jet_box(8)
    assert (m.n_elems, m.n_nodes) == (196608, 35937)
    assert np.isclose(tet_volumes6(m.xyz, m.tets).sum() / 6, 64.0)
    bc = jet_bc(m)
    assert not np.any(bc.dofs % 4 == 3)          # traction-free elsewhere: no pressure pin
    nodes = np.unique(bc.dofs // 4)
    wall = np.nonzero(np.abs(m.xyz[:, 0]) < 1e-12)[0]
    assert np.array_equal(nodes, wall) and bc.n == 3 * wall.size
    vals = bc.values.reshape(-1, 3)               # dofs sorted: node by node, components 0..2
    assert np.all(vals[:, 1:] == 0.0)
    r2 = m.xyz[nodes, 1] ** 2 + m.xyz[nodes, 2] ** 2
    inside = r2 < 0.25
    assert np.allclose(vals[inside, 0], 1.0 - 4.0 * r2[inside])
    assert np.all(vals[~inside, 0] == 0.0)
    assert vals[:, 0].max() == 1.0 and inside.sum() == 45   # grid nodes strictly inside r = 1/2, h = 1/8


def test_jitter_valid_and_seeded():
    a = jittered_cube(8, seed=0)
    b = jittered_cube(8, seed=0)
    c = jittered_cube(8, seed=1)
    assert np.array_equal(a.xyz, b.xyz) and not np.array_equal(a.xyz, c.xyz)
    assert a.meta["min_6V_over_h3"] > 0
    bnd = boundary_nodes(a.tets, a.n_nodes)
    ref = cavity_mesh(8)
    assert np.array_equal(a.xyz[bnd], ref.xyz[bnd])
    d = np.abs(a.xyz - ref.xyz).max()
    assert 0.1 / 8 < d <= 0.2 / 8


def test_cavity_bc():
    m = cavity_mesh(4)
    bc = cavity_bc(m)
    assert bc.n == 3 * (125 - 27) + 1
    assert np.sum(bc.values == 1.0) == 9        # open lid face only
    pin = bc.dofs[bc.dofs % 4 == 3]
    assert pin.size == 1 and np.allclose(m.xyz[pin[0] // 4], 0.5)


def test_paper_table1_fine_dofs_are_three_per_element():
    rows = []
    with open(os.path.join(GOLDEN, "table1_mesh_dofs.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, coarse, fine, total = line.split()
                rows.append((name, int(coarse), int(fine), int(total)))
    assert len(rows) == 5
    for name, coarse, fine, total in rows:
        assert coarse + fine == total, name
        assert fine % 3 == 0, name
    # the same bookkeeping on a generated mesh: 3 fine dofs per tet
    m = cavity_mesh(3)
    assert 3 * m.n_elems == 3 * 6 * 27


def _fd(f, x, i, h=1e-4):
    e = np.zeros(3)
    e[i] = h
    return (-f(x + 2 * e) + 8 * f(x + e) - 8 * f(x - e) + f(x - 2 * e)) / (12 * h)


def test_ethier_steinman_solves_navier_stokes():
    nu_l = 0.3
    rng = np.random.default_rng(0)
    t = 0.4
    for x in rng.uniform(-1, 1, size=(5, 3)):
        def U(p, tt=t):
            return np.array(es_velocity(p[0], p[1], p[2], tt, nu_l))

        def P(p):
            return es_pressure(p[0], p[1], p[2], t, nu_l)
        grad = np.stack([_fd(U, x, j) for j in range(3)], axis=1)     # grad[i, j] = d u_i / d x_j
        div = np.trace(grad)
        lap = np.zeros(3)
        h = 1e-3
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            lap += (U(x + e) - 2 * U(x) + U(x - e)) / h ** 2
        dudt = (U(x, t + 1e-5) - U(x, t - 1e-5)) / 2e-5
        gp = np.array([_fd(lambda p: np.array(P(p)), x, j) for j in range(3)])
        mom = dudt + grad @ U(x) - nu_l * lap + gp
        assert abs(div) < 1e-8
        assert np.max(np.abs(mom)) < 1e-5
        assert np.isclose(P(x), -0.5 * np.sum(U(x) ** 2), rtol=1e-12)


def test_configs_are_consistent():
    assert set(CONFIGS) == {"cavity4", "cavity32", "es64", "bfs8", "bfs16", "jet8"}
    assert CONFIGS["jet8"].re == 1000.0 and CONFIGS["jet8"].dt == 0.01
    assert CONFIGS["es64"].dt == 0.01 and CONFIGS["es64"].steps == 10
    assert CONFIGS["bfs16"].steps == 50
