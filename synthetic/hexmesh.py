"""Seeded general hexahedral meshes (vertex coordinates and cell vertex ids).

Only connectivity and coordinates are produced here, never finite element
quantities: cells list their 8 vertex ids in lexicographic local order
(local vertex v = bx + 2 by + 4 bz at reference corner (bx, by, bz)), and a
cell is positively oriented when x, y, z increase with bx, by, bz.
"""

from __future__ import annotations

import itertools

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree


def box_cells(nx: int, ny: int, nz: int) -> np.ndarray:
    """[nx*ny*nz, 8] int32 vertex ids of the cells of an ``nx x ny x nz`` box whose
    vertices are numbered x fastest (the order of ``box_vertices``); cells in
    x-fastest order."""
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    v = np.arange(8)
    bx, by, bz = v & 1, (v >> 1) & 1, v >> 2
    ids = (ex[:, None] + bx) + (nx + 1) * ((ey[:, None] + by) + (ny + 1) * (ez[:, None] + bz))
    return np.ascontiguousarray(ids.astype(np.int32))


def cube_rotations() -> list:
    """The 24 orientation-preserving symmetries of the reference cube, each as
    a permutation ``perm`` of the 8 local vertices: a rotated cell lists its
    vertices as ``old[perm]``."""
    out = []
    for axes in itertools.permutations(range(3)):
        sign = np.linalg.det(np.eye(3)[list(axes)])
        for flips in itertools.product((0, 1), repeat=3):
            if sign * (-1) ** sum(flips) < 0:
                continue
            perm = []
            for v in range(8):
                c = (v & 1, (v >> 1) & 1, v >> 2)          # new corner bits
                b = [c[axes[d]] ^ flips[d] for d in range(3)]  # old corner bits
                perm.append(b[0] + 2 * b[1] + 4 * b[2])
            out.append(np.array(perm))
    assert len(out) == 24
    return out


def relabel(vertices: np.ndarray, cells: np.ndarray, rng: np.random.Generator,
            rotate: bool = True, shuffle_vertices: bool = True, shuffle_cells: bool = False):
    """The same mesh with a random vertex numbering, every cell's local
    vertex order replaced by a random rotation of it, and optionally the cells
    permuted.  Returns (vertices, cells int32, vertex_perm, cell_perm) with
    new vertex i = old vertex vertex_perm[i] and new cell e = old cell
    cell_perm[e]."""
    vertices = np.asarray(vertices, dtype=np.float64)
    cells = np.asarray(cells, dtype=np.int64)
    nv, ne = vertices.shape[0], cells.shape[0]
    vp = rng.permutation(nv) if shuffle_vertices else np.arange(nv)
    inv = np.empty(nv, dtype=np.int64)
    inv[vp] = np.arange(nv)
    new_cells = inv[cells]
    if rotate:
        rots = cube_rotations()
        pick = rng.integers(0, 24, size=ne)
        new_cells = np.stack([new_cells[e, rots[pick[e]]] for e in range(ne)])
    cp = rng.permutation(ne) if shuffle_cells else np.arange(ne)
    new_cells = new_cells[cp]
    return (np.ascontiguousarray(vertices[vp]), np.ascontiguousarray(new_cells.astype(np.int32)), vp, cp)


def cube_in_cube(m: int, inner: float = 0.3, jitter: float = 0.0,
                 rng: np.random.Generator | None = None):
    """Unstructured hexahedral mesh of the unit cube: a central cube
    [inner, 1-inner]^3 surrounded by six hexahedral shells, one per face,
    each of the seven blocks split trilinearly into m^3 cells.  The corners
    of the central cube are shared by four blocks (a valence no structured
    box has).  With ``jitter`` > 0 every vertex off the outer boundary moves
    by U[-jitter*h, jitter*h] per coordinate, h = the smallest block spacing.
    Returns (vertices [nv, 3] float64, cells [7 m^3, 8] int32)."""
    a = float(inner)
    outer = lambda b: np.array(b, dtype=np.float64)
    inn = lambda b: a + (1.0 - 2.0 * a) * np.array(b, dtype=np.float64)
    blocks = [[inn(((v & 1), (v >> 1) & 1, v >> 2)) for v in range(8)]]
    for d in range(3):
        for side in (0, 1):
            corners = []
            for v in range(8):
                bits = [v & 1, (v >> 1) & 1, v >> 2]
                face = list(bits)
                face[d] = side
                # along d the shell runs from the outer face to the inner one
                # (side 0) or from the inner face to the outer one (side 1)
                use_inner = bits[d] == 1 if side == 0 else bits[d] == 0
                corners.append(inn(face) if use_inner else outer(face))
            blocks.append(corners)
    t = np.linspace(0.0, 1.0, m + 1)
    s3 = np.stack(np.meshgrid(t, t, t, indexing="ij")[::-1], axis=-1).reshape(-1, 3)   # x fastest
    bits = np.array([[v & 1, (v >> 1) & 1, v >> 2] for v in range(8)])
    shape = np.prod(np.where(bits[None, :, :] == 1, s3[:, None, :], 1.0 - s3[:, None, :]), axis=2)
    pts = np.concatenate([shape @ np.array(X) for X in blocks])          # [7 (m+1)^3, 3]
    # vertices shared by neighbouring blocks coincide up to rounding: merge
    # points closer than 1e-9 (the spacing is >= (1 - 2 inner) / m)
    pairs = cKDTree(pts).query_pairs(1e-9, output_type="ndarray")
    graph = coo_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(len(pts), len(pts)))
    _, label = connected_components(graph, directed=False)
    _, first, ids = np.unique(label, return_index=True, return_inverse=True)
    order = np.argsort(first)          # number vertices in order of first appearance
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    ids = rank[ids.reshape(-1)]
    verts = pts[first[order]]
    kk, jj, ii = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    base = (ii + (m + 1) * (jj + (m + 1) * kk)).reshape(-1)             # cell's (0,0,0) corner
    off = np.array([bx + (m + 1) * (by + (m + 1) * bz) for bx, by, bz in bits])
    local = base[:, None] + off[None, :]                                 # [m^3, 8]
    npb = (m + 1) ** 3
    cells = np.concatenate([ids[b * npb + local] for b in range(len(blocks))])
    if jitter > 0.0:
        if rng is None:
            raise ValueError("jitter needs a random generator")
        h = min(a, 1.0 - 2.0 * a) / m
        on_bnd = np.any((np.abs(verts) < 1e-12) | (np.abs(verts - 1.0) < 1e-12), axis=1)
        noise = rng.uniform(-1.0, 1.0, size=verts.shape) * (jitter * h)
        verts[~on_bnd] += noise[~on_bnd]
    return np.ascontiguousarray(verts), np.ascontiguousarray(np.array(cells, dtype=np.int32))


def sine_field(points: np.ndarray, amplitude: float, rng: np.random.Generator,
               n_modes: int = 3, kmax: int = 3) -> np.ndarray:
    """Nodal vector [3 * len(points)] of random product-sine modes evaluated at
    ``points``: u_c = A sum_m a[m,c] prod_d sin(pi k[m,d] s_d + phi[m,d]),
    s = the point's coordinates scaled to the bounding box, with the draws of
    ``sine_displacement``."""
    k = rng.integers(1, kmax + 1, size=(n_modes, 3))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=(n_modes, 3))
    a = rng.uniform(-1.0, 1.0, size=(n_modes, 3))
    x = np.asarray(points, dtype=np.float64)
    lo, hi = x.min(axis=0), x.max(axis=0)
    s = (x - lo) / np.where(hi > lo, hi - lo, 1.0)
    u = np.zeros((x.shape[0], 3))
    for mm in range(n_modes):
        f = np.prod(np.sin(np.pi * k[mm][None, :] * s + phi[mm][None, :]), axis=1)
        u += f[:, None] * a[mm][None, :]
    return np.ascontiguousarray((amplitude * u).reshape(-1))
