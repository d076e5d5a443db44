"""Tetrahedral mesh generators (Kuhn split of structured boxes).

Every generator returns positively oriented linear tetrahedra.  The paper
runs on unstructured tetrahedral meshes (Introduction; Section 6); these
synthetic stand-ins reproduce their structure: linear tets, about 24 tets
per interior node and 15 node neighbours, and for the jittered cube a
random perturbation of the interior nodes.

Layouts (host numpy arrays):
  xyz   float64 [n_nodes, 3]
  tets  int32   [n_elems, 4]   vertex ids, det[x1-x0, x2-x0, x3-x0] > 0
Numbering: nodes and cells are numbered brick by brick (bricks of 4x4x4
lattice points, bricks in lexicographic order, points inside a brick
lexicographic with k fastest), restricted to the nodes that active cells
touch; six tets per cell.  Contiguous ranges of node ids are then compact
groups of nodes, which the GPU library's tiled assembly and SpMV exploit.
order="lex" gives plain lexicographic numbering instead.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import permutations

import numpy as np


@dataclass
class Mesh:
    xyz: np.ndarray           # float64 [n_nodes, 3]
    tets: np.ndarray          # int32 [n_elems, 4]
    name: str = "mesh"
    h: float = 0.0            # nominal cell size (smallest lattice spacing)
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.tets.shape[0])


def _kuhn_offsets():
    """Six Kuhn tets of the unit cube: paths 0 -> e_p0 -> e_p0+e_p1 -> (1,1,1).

    Odd permutations produce negatively oriented tets; their last two
    vertices are swapped so that every tet is positively oriented.
    """
    tets = []
    for perm in permutations(range(3)):
        v = [np.zeros(3, dtype=np.int64)]
        for ax in perm:
            nxt = v[-1].copy()
            nxt[ax] += 1
            v.append(nxt)
        m = np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]], axis=1)
        if np.linalg.det(m) < 0:
            v[2], v[3] = v[3], v[2]
        tets.append(np.stack(v))
    return np.stack(tets)      # [6, 4, 3] integer corner offsets


BRICK = 4


def _brick_key(i, j, k, brick=BRICK):
    """Sort key: brick index (lexicographic), then position inside the brick."""
    bi, bj, bk = i // brick, j // brick, k // brick
    big = 1 << 20
    return (((bi * big + bj) * big + bk) * brick + i % brick) * brick * brick + (j % brick) * brick + k % brick


def kuhn_box(shape, lo, hi, cell_mask=None, name="box", order="brick") -> Mesh:
    """Kuhn split of an (nx, ny, nz) lattice of cells spanning [lo, hi].

    cell_mask (bool [nx, ny, nz]) selects active cells; nodes not touched by
    any active cell are dropped and the rest numbered in `order`.
    """
    nx, ny, nz = (int(s) for s in shape)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    if cell_mask is None:
        cell_mask = np.ones((nx, ny, nz), dtype=bool)
    offs = _kuhn_offsets()

    ci, cj, ck = np.nonzero(cell_mask)          # lexicographic, k fastest
    if order == "brick":
        perm = np.argsort(_brick_key(ci, cj, ck), kind="stable")
        ci, cj, ck = ci[perm], cj[perm], ck[perm]
    corner = np.stack([ci, cj, ck], axis=1)     # [n_cells, 3]
    # lattice coordinates of the 6x4 vertices of each cell
    lat = corner[:, None, None, :] + offs[None, :, :, :]          # [nc, 6, 4, 3]
    lat = lat.reshape(-1, 4, 3)
    lin = (lat[..., 0] * (ny + 1) + lat[..., 1]) * (nz + 1) + lat[..., 2]

    used = np.zeros((nx + 1) * (ny + 1) * (nz + 1), dtype=bool)
    used[lin.ravel()] = True
    idx = np.nonzero(used)[0]                   # lexicographic lattice ids of the nodes
    i = idx // ((ny + 1) * (nz + 1))
    j = (idx // (nz + 1)) % (ny + 1)
    k = idx % (nz + 1)
    if order == "brick":
        perm = np.argsort(_brick_key(i, j, k), kind="stable")
        idx, i, j, k = idx[perm], i[perm], j[perm], k[perm]
    new_id = -np.ones(used.size, dtype=np.int64)
    new_id[idx] = np.arange(idx.size)
    tets = new_id[lin].astype(np.int32)
    step = (hi - lo) / np.array([nx, ny, nz], dtype=np.float64)
    xyz = np.stack([lo[0] + i * step[0], lo[1] + j * step[1], lo[2] + k * step[2]], axis=1)
    mesh = Mesh(xyz=np.ascontiguousarray(xyz), tets=np.ascontiguousarray(tets),
                name=name, h=float(step.min()),
                meta={"lattice": (nx, ny, nz), "lattice_index": np.stack([i, j, k], axis=1)})
    _assert_positive(mesh)
    return mesh


def tet_volumes6(xyz, tets):
    """6 x signed volume of each tet (det of the edge matrix)."""
    x0 = xyz[tets[:, 0]]
    e1 = xyz[tets[:, 1]] - x0
    e2 = xyz[tets[:, 2]] - x0
    e3 = xyz[tets[:, 3]] - x0
    return np.einsum("ei,ei->e", e1, np.cross(e2, e3))


def _assert_positive(mesh: Mesh):
    v6 = tet_volumes6(mesh.xyz, mesh.tets)
    if not np.all(v6 > 0):
        bad = int(np.argmin(v6))
        raise ValueError(f"{mesh.name}: tet {bad} has det J = {v6[bad]:.3e} <= 0")


def cavity_mesh(n: int) -> Mesh:
    """Unit cube [0,1]^3, n^3 cells x 6 tets (lid-driven cavity)."""
    return kuhn_box((n, n, n), (0, 0, 0), (1, 1, 1), name=f"cavity{n}")


def jittered_cube(n: int, seed: int = 0, amp: float = 0.2) -> Mesh:
    """Unit cube with every interior node displaced by U(-amp*h, amp*h) per coordinate.

    The displacements are drawn for all lattice nodes in lexicographic lattice
    order (k fastest) from numpy.random.default_rng(seed), whatever the node
    numbering, and applied only to interior nodes, so the boundary stays planar.
    """
    m = kuhn_box((n, n, n), (0, 0, 0), (1, 1, 1), name=f"jitter{n}_s{seed}")
    h = 1.0 / n
    rng = np.random.default_rng(seed)
    lat = m.meta["lattice_index"]
    d_lex = rng.uniform(-amp * h, amp * h, size=((n + 1) ** 3, 3))
    d = d_lex[(lat[:, 0] * (n + 1) + lat[:, 1]) * (n + 1) + lat[:, 2]]
    interior = np.all((lat > 0) & (lat < n), axis=1)
    m.xyz = m.xyz + d * interior[:, None]
    m.meta["seed"] = seed
    _assert_positive(m)
    v6 = tet_volumes6(m.xyz, m.tets)
    m.meta["min_6V_over_h3"] = float(v6.min() / h ** 3)
    return m


def jitter_interior(mesh: Mesh, amp: float, seed: int) -> Mesh:
    """Displace every node off the boundary by U(-amp*h, amp*h) per coordinate
    (numpy.random.default_rng(seed), drawn for all nodes in node order)."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(-amp * mesh.h, amp * mesh.h, size=(mesh.n_nodes, 3))
    inner = ~boundary_nodes(mesh.tets, mesh.n_nodes)
    out = Mesh(xyz=mesh.xyz + d * inner[:, None], tets=mesh.tets, name=mesh.name + f"_j{seed}",
               h=mesh.h, meta=dict(mesh.meta))
    _assert_positive(out)
    return out


def backward_facing_step(cx: int, cy: int, cz: int) -> Mesh:
    """Backward-facing-step channel: step height 1, expansion ratio 2.

    Inlet channel x in [-5, 0], y in [1, 2]; outlet channel x in [0, 30],
    y in [0, 2]; span z in [0, 4].  (cx, cy, cz) are cells per unit length.
    """
    nx, ny, nz = 35 * cx, 2 * cy, 4 * cz
    i = np.arange(nx)[:, None, None]
    j = np.arange(ny)[None, :, None]
    mask = np.broadcast_to((i >= 5 * cx) | (j >= cy), (nx, ny, nz))
    return kuhn_box((nx, ny, nz), (-5, 0, 0), (30, 2, 4), cell_mask=np.array(mask),
                    name=f"bfs_{cx}_{cy}_{cz}")


def jet_box(c: int) -> Mesh:
    """Jet from an orifice: the box x in [0, 4], y, z in [-2, 2] with c cells per unit
    length (4c x 4c x 4c cells x 6 tets).  The orifice (diameter 1) is centred at the
    origin, in the wall x = 0."""
    n = 4 * c
    return kuhn_box((n, n, n), (0, -2, -2), (4, 2, 2), name=f"jet_{c}")


def boundary_nodes(tets: np.ndarray, n_nodes: int) -> np.ndarray:
    """Bool mask of nodes lying on a boundary face (a face owned by one tet)."""
    faces = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]],
                            tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    faces = np.sort(faces, axis=1).astype(np.int64)
    key = (faces[:, 0] * n_nodes + faces[:, 1]) * n_nodes + faces[:, 2]
    uniq, cnt = np.unique(key, return_counts=True)
    bkey = uniq[cnt == 1]
    mask = np.zeros(n_nodes, dtype=bool)
    a = bkey // (n_nodes * n_nodes)
    b = (bkey // n_nodes) % n_nodes
    c = bkey % n_nodes
    mask[a] = True
    mask[b] = True
    mask[c] = True
    return mask


def count_edges(tets: np.ndarray, n_nodes: int) -> int:
    pairs = np.concatenate([tets[:, [a, b]] for a in range(4) for b in range(a + 1, 4)])
    pairs = np.sort(pairs, axis=1).astype(np.int64)
    return int(np.unique(pairs[:, 0] * n_nodes + pairs[:, 1]).size)
