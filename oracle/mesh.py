"""Structured Q_p box mesh: numbering, trilinear geometry, physical gradients.

The cell-wise quadrature of Sec. 2.4 needs, at every quadrature point, the
reference-to-physical Jacobian J_g, its determinant (the "J_q" factor of the
cell integral) and the physical basis gradients Grad N_a = J_g^{-T} dN_a/dxi.
The geometry map is the trilinear (Q1) map through the 8 cell vertices.

Numbering (the public layout of the library): nodes of a degree-p
``nx x ny x nz`` box are (I, J, K) with I in [0, p*nx], numbered
I + Nx*(J + Ny*K) (Nx = p*nx+1); node ``n`` carries dofs 3n, 3n+1, 3n+2.
Cells are numbered ex + nx*(ey + ny*ez); cell-local node (i, j, k) is global
node (p*ex+i, p*ey+j, p*ez+k).
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


class BoxMesh:
    """Degree-p box mesh with corner vertices ``vertices`` [(nx+1)(ny+1)(nz+1), 3]."""

    def __init__(self, nx: int, ny: int, nz: int, degree: int, vertices: np.ndarray):
        self.nx, self.ny, self.nz, self.degree = int(nx), int(ny), int(nz), int(degree)
        p = self.degree
        self.vertices = np.asarray(vertices, dtype=np.float64).reshape(-1, 3)
        if self.vertices.shape[0] != (nx + 1) * (ny + 1) * (nz + 1):
            raise ValueError("vertex array has the wrong length")
        self.basis = TensorBasis(p)
        self.n = p + 1
        self.nodes_per_dir = (p * nx + 1, p * ny + 1, p * nz + 1)
        self.n_nodes = int(np.prod(self.nodes_per_dir))
        self.n_dofs = 3 * self.n_nodes
        self.n_elems = nx * ny * nz
        self.nq3 = self.basis.nq ** 3
        self.n3 = self.n ** 3
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

    def node_positions(self) -> np.ndarray:
        """Physical coordinates [n_nodes, 3] of the Q_p support points (trilinear map
        of the Gauss-Lobatto reference points)."""
        n = self.n
        t = self.basis.nodes_1d
        kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        ref = np.stack([t[ii.ravel()], t[jj.ravel()], t[kk.ravel()]], axis=1)  # [n3, 3]
        vals, _ = trilinear_shape(ref)                                           # [n3, 8]
        X = self.vertices[self.elem_vertices]                                    # [ne, 8, 3]
        pos = np.einsum("av,evd->ead", vals, X)
        out = np.zeros((self.n_nodes, 3))
        out[self.elem_nodes.ravel()] = pos.reshape(-1, 3)
        return out

    def elem_dofs(self, elems=None) -> np.ndarray:
        """dof[e, c, a] = 3 * node(e, a) + c."""
        elems = np.arange(self.n_elems) if elems is None else np.asarray(elems)
        nodes = self.elem_nodes[elems]
        return 3 * nodes[:, None, :] + np.arange(3)[None, :, None]

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
