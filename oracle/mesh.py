"""Q_p hexahedral meshes: numbering, trilinear geometry, physical gradients.

The cell-wise quadrature of Sec. 2.4 needs, at every quadrature point, the
reference-to-physical Jacobian J_g, its determinant (the "J_q" factor of the
cell integral) and the physical basis gradients Grad N_a = J_g^{-T} dN_a/dxi.
The geometry map is the trilinear (Q1) map through the 8 cell vertices.

Numbering (the public layout of the library): nodes of a degree-p
``nx x ny x nz`` box are (I, J, K) with I in [0, p*nx], numbered
I + Nx*(J + Ny*K) (Nx = p*nx+1); node ``n`` carries dofs 3n, 3n+1, 3n+2.
Cells are numbered ex + nx*(ey + ny*ez); cell-local node (i, j, k) is global
node (p*ex+i, p*ey+j, p*ez+k).

General hexahedral meshes (``HexMesh``) are given by vertex coordinates and
the 8 vertex ids of every cell in lexicographic order (local vertex
v = bx + 2 by + 4 bz sits at reference corner (bx, by, bz)).  Their Q_p nodes
follow the library's canonical numbering, which depends only on the vertex
ids:

1. node v < nv is mesh vertex v;
2. (p >= 2) the unique edges, sorted by their (lower id, higher id) vertex
   pair, own p-1 nodes each, numbered in order of their distance from the
   lower-id end;
3. the unique faces, sorted by their ascending 4-tuple of vertex ids, own
   (p-1)^2 nodes each, (s-1) + (p-1)(t-1): the face is walked from its
   lowest-id vertex o, s counting support points towards the lower-id of o's
   two edge neighbours on the face and t towards the other;
4. every cell owns (p-1)^3 interior nodes in its local lexicographic order,
   cells in order.
"""

from __future__ import annotations

import numpy as np

from .basis import TensorBasis


def trilinear_shape(xi: np.ndarray):
    """Values [.., 8] and reference gradients [.., 8, 3] of the 8 trilinear
    vertex functions N1_v(xi) = prod_d (xi_d if bit_d(v) else 1 - xi_d),
    v = vx + 2*vy + 4*vz."""
    xi = np.asarray(xi, dtype=np.float64)
    vals = np.ones(xi.shape[:-1] + (8,))
    grads = np.ones(xi.shape[:-1] + (8, 3))
    for v in range(8):
        bits = (v & 1, (v >> 1) & 1, (v >> 2) & 1)
        f = [xi[..., d] if bits[d] else 1.0 - xi[..., d] for d in range(3)]
        df = [1.0 if bits[d] else -1.0 for d in range(3)]
        vals[..., v] = f[0] * f[1] * f[2]
        grads[..., v, 0] = df[0] * f[1] * f[2]
        grads[..., v, 1] = f[0] * df[1] * f[2]
        grads[..., v, 2] = f[0] * f[1] * df[2]
    return vals, grads


class _TrilinearCells:
    """Geometry of cells mapped trilinearly from their 8 vertices; subclasses
    set vertices, elem_vertices, elem_nodes, basis, degree, n, n3, nq3,
    n_nodes, n_dofs, n_elems and _tri_vals/_tri_grads."""

    def _init_basis(self, degree):
        self.degree = int(degree)
        self.basis = TensorBasis(self.degree)
        self.n = self.degree + 1
        self.n3 = self.n ** 3
        self.nq3 = self.basis.nq ** 3
        self._tri_vals, self._tri_grads = trilinear_shape(self.basis.points)  # [nq3,8], [nq3,8,3]

    # ------------------------------------------------------------------ geometry
    def jacobians(self, elems=None) -> np.ndarray:
        """J_g[e, q, d, A] = dX_d / dxi_A at each quadrature point (trilinear map)."""
        elems = np.arange(self.n_elems) if elems is None else np.asarray(elems)
        X = self.vertices[self.elem_vertices[elems]]               # [E, 8, 3]
        return np.einsum("evd,qvA->eqdA", X, self._tri_grads)

    def geometry(self, elems=None):
        """Physical basis gradients and integration weights for cells ``elems``.

        Returns ``gradN[e, q, a, A] = sum_B (J_g^{-1})_{B A} dN_a/dxi_B`` and
        ``JxW[e, q] = w_q * det J_g``.  Raises if det J_g <= 0 anywhere.
        """
        Jg = self.jacobians(elems)
        det = np.linalg.det(Jg)
        if np.any(det <= 0.0):
            raise ValueError("inverted or degenerate cell geometry (det J_g <= 0)")
        Jinv = np.linalg.inv(Jg)                                     # [E, q, A, d]
        gradN = np.einsum("eqBA,qaB->eqaA", Jinv, self.basis.grads)
        JxW = det * self.basis.weights[None, :]
        return gradN, JxW

    def cell_node_positions(self) -> np.ndarray:
        """[ne, n3, 3]: every cell's trilinear image of its Gauss-Lobatto
        reference support points, local node a = i + n(j + n k)."""
        n = self.n
        t = self.basis.nodes_1d
        kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        ref = np.stack([t[ii.ravel()], t[jj.ravel()], t[kk.ravel()]], axis=1)  # [n3, 3]
        vals, _ = trilinear_shape(ref)                                           # [n3, 8]
        X = self.vertices[self.elem_vertices]                                    # [ne, 8, 3]
        return np.einsum("av,evd->ead", vals, X)

    def node_positions(self) -> np.ndarray:
        """Physical coordinates [n_nodes, 3] of the Q_p support points (trilinear map
        of the Gauss-Lobatto reference points)."""
        out = np.zeros((self.n_nodes, 3))
        out[self.elem_nodes.ravel()] = self.cell_node_positions().reshape(-1, 3)
        return out

    def elem_dofs(self, elems=None) -> np.ndarray:
        """dof[e, c, a] = 3 * node(e, a) + c."""
        elems = np.arange(self.n_elems) if elems is None else np.asarray(elems)
        nodes = self.elem_nodes[elems]
        return 3 * nodes[:, None, :] + np.arange(3)[None, :, None]


class BoxMesh(_TrilinearCells):
    """Degree-p box mesh with corner vertices ``vertices`` [(nx+1)(ny+1)(nz+1), 3]."""

    def __init__(self, nx: int, ny: int, nz: int, degree: int, vertices: np.ndarray):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self._init_basis(degree)
        p = self.degree
        self.vertices = np.asarray(vertices, dtype=np.float64).reshape(-1, 3)
        if self.vertices.shape[0] != (nx + 1) * (ny + 1) * (nz + 1):
            raise ValueError("vertex array has the wrong length")
        self.nodes_per_dir = (p * nx + 1, p * ny + 1, p * nz + 1)
        self.n_nodes = int(np.prod(self.nodes_per_dir))
        self.n_dofs = 3 * self.n_nodes
        self.n_elems = nx * ny * nz
        # connectivity
        Nx, Ny, _ = self.nodes_per_dir
        ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
        n = self.n
        kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()   # local node a = i + n(j + n k)
        I = p * ex[:, None] + ii[None, :]
        J = p * ey[:, None] + jj[None, :]
        K = p * ez[:, None] + kk[None, :]
        self.elem_nodes = I + Nx * (J + Ny * K)          # [ne, n3]
        vx = np.array([v & 1 for v in range(8)])
        vy = np.array([(v >> 1) & 1 for v in range(8)])
        vz = np.array([(v >> 2) & 1 for v in range(8)])
        vid = (ex[:, None] + vx) + (nx + 1) * ((ey[:, None] + vy) + (ny + 1) * (ez[:, None] + vz))
        self.elem_vertices = vid                         # [ne, 8]

    def boundary_nodes(self) -> np.ndarray:
        """Boolean mask [n_nodes]: node lies on the box boundary."""
        Nx, Ny, Nz = self.nodes_per_dir
        K, J, I = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
        b = (I == 0) | (I == Nx - 1) | (J == 0) | (J == Ny - 1) | (K == 0) | (K == Nz - 1)
        return b.ravel()

    def elements_of_nodes(self, nodes) -> np.ndarray:
        """Sorted unique cells that touch any of ``nodes``."""
        nodes = np.atleast_1d(np.asarray(nodes))
        p = self.degree
        Nx, Ny, _ = self.nodes_per_dir
        I, J, K = nodes % Nx, (nodes // Nx) % Ny, nodes // (Nx * Ny)
        cells = []
        for I0, J0, K0 in zip(I, J, K):
            exs = {min(max((I0 - s) // p, 0), self.nx - 1) for s in (0, 1)} if p > 0 else set()
            eys = {min(max((J0 - s) // p, 0), self.ny - 1) for s in (0, 1)}
            ezs = {min(max((K0 - s) // p, 0), self.nz - 1) for s in (0, 1)}
            # keep only cells whose node range actually contains the node
            for ex in exs:
                if not (p * ex <= I0 <= p * ex + p):
                    continue
                for ey in eys:
                    if not (p * ey <= J0 <= p * ey + p):
                        continue
                    for ez in ezs:
                        if p * ez <= K0 <= p * ez + p:
                            cells.append(ex + self.nx * (ey + self.ny * ez))
        return np.unique(np.array(cells, dtype=np.int64))


# Local vertices of the reference cube: v = bx + 2 by + 4 bz.
def _corner(b0, b1, b2):
    return b0 + 2 * b1 + 4 * b2


class HexMesh(_TrilinearCells):
    """Degree-p mesh of general hexahedra: ``vertices`` [nv, 3] and
    ``elem_vertices`` [ne, 8] (lexicographic local order), with the canonical
    node numbering of the module docstring."""

    def __init__(self, vertices, elem_vertices, degree: int):
        self._init_basis(degree)
        p = self.degree
        self.vertices = np.asarray(vertices, dtype=np.float64).reshape(-1, 3)
        ev = np.asarray(elem_vertices, dtype=np.int64).reshape(-1, 8)
        nv, ne = self.vertices.shape[0], ev.shape[0]
        if ne == 0 or ev.min() < 0 or ev.max() >= nv:
            raise ValueError("cell vertex ids out of range")
        if any(len(set(row)) != 8 for row in ev.tolist()):
            raise ValueError("a cell repeats a vertex")
        self.elem_vertices = ev
        self.n_elems = ne
        m = p - 1
        # entities of every cell, keyed by global vertex ids
        edges, faces = set(), {}
        for row in ev.tolist():
            for d in range(3):
                for v in range(8):
                    if not (v >> d) & 1:
                        a, b = row[v], row[v | (1 << d)]
                        edges.add((min(a, b), max(a, b)))
            for d in range(3):
                d1, d2 = [x for x in range(3) if x != d]
                for side in (0, 1):
                    key, _, path = self._face_walk(row, d, side, d1, d2)
                    prev = faces.setdefault(key, [path, 0])
                    if prev[0] != path:
                        raise ValueError(f"cells disagree on the edges of face {key}")
                    prev[1] += 1
                    if prev[1] > 2:
                        raise ValueError(f"face {key} belongs to more than two cells")
        edge_rank = {k: r for r, k in enumerate(sorted(edges))}
        face_rank = {k: r for r, k in enumerate(sorted(faces))}
        base_e = nv
        base_f = base_e + len(edge_rank) * m
        base_i = base_f + len(face_rank) * m * m
        self.n_edges, self.n_faces = len(edge_rank), len(face_rank)
        self.n_nodes = base_i + ne * m ** 3
        self.n_dofs = 3 * self.n_nodes
        n = self.n
        nodes = np.empty((ne, n ** 3), dtype=np.int64)
        for e, row in enumerate(ev.tolist()):
            for k in range(n):
                for j in range(n):
                    for i in range(n):
                        c = (i, j, k)
                        ends = [x in (0, p) for x in c]
                        a = i + n * (j + n * k)
                        if all(ends):
                            nodes[e, a] = row[_corner(*(x // p for x in c))]
                        elif sum(ends) == 2:
                            d = ends.index(False)
                            lo_bits = [x // p if x in (0, p) else 0 for x in c]
                            hi_bits = list(lo_bits)
                            hi_bits[d] = 1
                            ga, gb = row[_corner(*lo_bits)], row[_corner(*hi_bits)]
                            s = c[d] if ga < gb else p - c[d]
                            nodes[e, a] = base_e + edge_rank[(min(ga, gb), max(ga, gb))] * m + (s - 1)
                        elif sum(ends) == 1:
                            d = ends.index(True)
                            d1, d2 = [x for x in range(3) if x != d]
                            key, (o1, o2, first_is_d1), _ = self._face_walk(row, d, c[d] // p, d1, d2)
                            s1 = p - c[d1] if o1 else c[d1]
                            s2 = p - c[d2] if o2 else c[d2]
                            s, t = (s1, s2) if first_is_d1 else (s2, s1)
                            nodes[e, a] = base_f + face_rank[key] * m * m + (s - 1) + m * (t - 1)
                        else:
                            nodes[e, a] = base_i + e * m ** 3 + (i - 1) + m * ((j - 1) + m * (k - 1))
        self.elem_nodes = nodes

    @staticmethod
    def _face_walk(row, d, side, d1, d2):
        """(sorted vertex ids, (o1, o2, first_is_d1), path) of the cell face
        with reference coordinate d fixed at ``side``: (o1, o2) is the corner
        of the lowest-id vertex o in the face's (d1, d2) corner bits, the walk's
        first axis is d1 when the neighbour of o along d1 has the lower id, and
        path = (o, lower neighbour, higher neighbour, opposite corner) in global
        ids, which two cells sharing the face must agree on."""
        def gid(b1, b2):
            bits = [0, 0, 0]
            bits[d], bits[d1], bits[d2] = side, b1, b2
            return row[_corner(*bits)]
        ids = {(b1, b2): gid(b1, b2) for b1 in (0, 1) for b2 in (0, 1)}
        o1, o2 = min(ids, key=ids.get)
        n1, n2 = ids[(1 - o1, o2)], ids[(o1, 1 - o2)]
        key = tuple(sorted(ids.values()))
        walk = (o1, o2, n1 < n2)
        path = (ids[(o1, o2)], min(n1, n2), max(n1, n2), ids[(1 - o1, 1 - o2)])
        return key, walk, path

    def elements_of_nodes(self, nodes) -> np.ndarray:
        """Sorted unique cells that touch any of ``nodes``."""
        hit = np.isin(self.elem_nodes, np.atleast_1d(np.asarray(nodes))).any(axis=1)
        return np.nonzero(hit)[0]
