"""Seeded generators for box meshes, displacement states and test vectors.

Conventions shared by every consumer (they are the public data layout of the
library, not part of the method):

* mesh vertices of an ``nx x ny x nz`` box are stored as an array of shape
  ``((nx+1)*(ny+1)*(nz+1), 3)`` with the x index running fastest;
* a degree-``p`` box has ``(p*nx+1)*(p*ny+1)*(p*nz+1)`` nodes, numbered
  lexicographically with x fastest, and node ``n`` carries the three degrees
  of freedom ``3*n + c`` (``c`` = 0, 1, 2 for x, y, z);
* random streams come from ``numpy.random.default_rng([cfg_id, stream])`` with
  stream 0 for vertex jitter, 1 for the displacement modes and ``2 + k`` for
  the k-th test vector.
"""

from __future__ import annotations

import numpy as np


def rng_for(cfg_id: int, stream: int) -> np.random.Generator:
    """Independent, reproducible random stream ``stream`` of configuration ``cfg_id``."""
    return np.random.default_rng([int(cfg_id), int(stream)])


def box_counts(nx: int, ny: int, nz: int, degree: int) -> dict:
    """Element, node and DoF counts of a structured degree-``degree`` box."""
    nnx, nny, nnz = degree * nx + 1, degree * ny + 1, degree * nz + 1
    n_nodes = nnx * nny * nnz
    return {
        "n_elems": nx * ny * nz,
        "nodes_per_dir": (nnx, nny, nnz),
        "n_nodes": n_nodes,
        "n_dofs": 3 * n_nodes,
        "n_vertices": (nx + 1) * (ny + 1) * (nz + 1),
    }


def box_vertices(nx: int, ny: int, nz: int, lengths=(1.0, 1.0, 1.0),
                 jitter: float = 0.0, rng: np.random.Generator | None = None) -> np.ndarray:
    """Corner vertices of an ``nx x ny x nz`` box ``[0,Lx]x[0,Ly]x[0,Lz]``.

    With ``jitter > 0`` every *interior* vertex coordinate is moved by an
    independent uniform draw from ``[-jitter*h_d, +jitter*h_d]`` where ``h_d``
    is the element size along axis ``d``.  Boundary vertices stay on the box
    faces, so the domain remains exactly the box.
    Returns a C-contiguous float64 array ``((nx+1)*(ny+1)*(nz+1), 3)``, x fastest.
    """
    lx, ly, lz = (float(v) for v in lengths)
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    zs = np.linspace(0.0, lz, nz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float64)
    if jitter > 0.0:
        if rng is None:
            raise ValueError("jitter needs a random generator")
        h = np.array([lx / nx, ly / ny, lz / nz])
        noise = rng.uniform(-1.0, 1.0, size=verts.shape) * (jitter * h)
        iz, iy, ix = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                                 indexing="ij")
        interior = ((ix > 0) & (ix < nx) & (iy > 0) & (iy < ny) & (iz > 0) & (iz < nz)).ravel()
        verts[interior] += noise[interior]
    return np.ascontiguousarray(verts)


def sine_displacement(nx: int, ny: int, nz: int, degree: int, amplitude: float,
                      rng: np.random.Generator, n_modes: int = 3, kmax: int = 3) -> np.ndarray:
    """Nodal displacement vector made of ``n_modes`` random product-sine modes.

    ``u_c = A * sum_m a[m,c] * prod_d sin(pi * k[m,d] * s_d + phi[m,d])`` where
    ``s_d = I_d / (degree * n_d)`` is the node's logical (domain-normalised)
    coordinate, ``k ~ U{1..kmax}``, ``phi ~ U[0, 2 pi)`` and ``a ~ U[-1, 1]``.
    The field lives on the node grid only; it is a smooth set of nodal values,
    not a function of the (possibly jittered) physical positions.
    Returns float64 ``[3 * n_nodes]`` with dof = 3*node + c.
    """
    k = rng.integers(1, kmax + 1, size=(n_modes, 3))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=(n_modes, 3))
    a = rng.uniform(-1.0, 1.0, size=(n_modes, 3))
    nnx, nny, nnz = degree * nx + 1, degree * ny + 1, degree * nz + 1
    s = [np.arange(nnx) / (nnx - 1), np.arange(nny) / (nny - 1), np.arange(nnz) / (nnz - 1)]
    u = np.zeros((nnz, nny, nnx, 3))
    for m in range(n_modes):
        fx = np.sin(np.pi * k[m, 0] * s[0] + phi[m, 0])
        fy = np.sin(np.pi * k[m, 1] * s[1] + phi[m, 1])
        fz = np.sin(np.pi * k[m, 2] * s[2] + phi[m, 2])
        mode = fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
        u += mode[..., None] * a[m][None, None, None, :]
    return np.ascontiguousarray((amplitude * u).reshape(-1))


def random_vectors(n_dofs: int, count: int, rng: np.random.Generator) -> np.ndarray:
    """``count`` i.i.d. N(0,1) vectors of length ``n_dofs`` (float64, shape (count, n_dofs))."""
    return rng.standard_normal(size=(count, n_dofs))



def clamp_and_twist(nx: int, ny: int, nz: int, degree: int, lengths, theta: float):
    """Dirichlet data of the twisted beam: every dof of the nodes on the face
    x = 0 is 0; the nodes on the face x = Lx are rotated by ``theta`` about the
    beam axis through c = (Lx, Ly/2, Lz/2): u = R_x(theta) (X - c) - (X - c).

    Node positions are those of the undistorted box with equispaced nodes
    (degree <= 2, where Gauss-Lobatto and equispaced points coincide).
    Returns (dofs int64, values float64), dofs sorted.
    """
    if degree > 2:
        raise ValueError("twist data assumes equispaced nodes (degree <= 2)")
    lx, ly, lz = (float(v) for v in lengths)
    nnx, nny, nnz = degree * nx + 1, degree * ny + 1, degree * nz + 1
    J, K = np.meshgrid(np.arange(nny), np.arange(nnz), indexing="ij")
    J, K = J.ravel(), K.ravel()
    left = 0 + nnx * (J + nny * K)
    right = (nnx - 1) + nnx * (J + nny * K)
    y = J * (ly / (nny - 1)) - 0.5 * ly
    z = K * (lz / (nnz - 1)) - 0.5 * lz
    c, s = np.cos(theta), np.sin(theta)
    uy = (c * y - s * z) - y
    uz = (s * y + c * z) - z
    dofs = np.concatenate([3 * left[:, None] + np.arange(3), 3 * right[:, None] + np.arange(3)]).ravel()
    vals = np.concatenate([np.zeros((left.size, 3)), np.stack([np.zeros_like(uy), uy, uz], axis=1)]).ravel()
    order = np.argsort(dofs)
    return dofs[order].astype(np.int64), vals[order]
