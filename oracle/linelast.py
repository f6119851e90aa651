"""Textbook small-strain stiffness K = sum_q JxW B^T D B (isotropic, Voigt).

Independent of the finite-strain code paths: used only to pin the u = 0 limit
of the tangent (the linearisation of eq. DF at F = I is linear elasticity).
Voigt order (xx, yy, zz, yz, xz, xy) with engineering shear strains.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import BoxMesh


def isotropic_D(lam_lin: float, mu: float) -> np.ndarray:
    D = np.zeros((6, 6))
    D[:3, :3] = lam_lin
    D[0, 0] = D[1, 1] = D[2, 2] = lam_lin + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def strain_displacement(gradN: np.ndarray) -> np.ndarray:
    """B[..., 6, 3, n3] from physical basis gradients gradN[..., n3, 3];
    column (c, a) is the displacement component c of node a."""
    shp = gradN.shape[:-2]
    n3 = gradN.shape[-2]
    B = np.zeros(shp + (6, 3, n3))
    Nx, Ny, Nz = gradN[..., 0], gradN[..., 1], gradN[..., 2]
    B[..., 0, 0, :] = Nx
    B[..., 1, 1, :] = Ny
    B[..., 2, 2, :] = Nz
    B[..., 3, 1, :] = Nz
    B[..., 3, 2, :] = Ny
    B[..., 4, 0, :] = Nz
    B[..., 4, 2, :] = Nx
    B[..., 5, 0, :] = Ny
    B[..., 5, 1, :] = Nx
    return B


def assemble(mesh: BoxMesh, lam_lin: float, mu: float) -> sp.csr_matrix:
    D = isotropic_D(lam_lin, mu)
    gradN, JxW = mesh.geometry()
    B = strain_displacement(gradN).reshape(gradN.shape[0], gradN.shape[1], 6, -1)   # [E,q,6,3*n3]
    Ke = np.einsum("eq,eqsm,st,eqtn->emn", JxW, B, D, B)
    d = mesh.elem_dofs().reshape(mesh.n_elems, -1)
    m = d.shape[1]
    rows = np.repeat(d, m, axis=1).ravel()
    cols = np.tile(d, (1, m)).ravel()
    K = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(mesh.n_dofs, mesh.n_dofs)).tocsr()
    K.sum_duplicates()
    return K
