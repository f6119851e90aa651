"""Discrete residual, energy and tangent of the hyperelastic problem.

Definitions followed (paper Sec. 2.1-2.4):

* energy   E(u)      = sum_cells sum_q JxW_q Psi(F_q)                       (energy functional, no traction term)
* residual R_(a,i)   = sum_cells sum_q JxW_q P_iA(F_q) Grad_A N_a            (weak form F, eq. F, tested with phi = N_a e_i)
* tangent  v_(a,i)   = sum_cells sum_q JxW_q Grad_A N_a L_iAjB(F_q) H_jB      (eq. DF with the cell quadrature of Sec. 2.4)
           H_jB      = sum_b w_(b,j) Grad_B N_b                            (Grad of the input field)

with F_q = I + sum_a u_(a) (x) Grad N_a(x_q).  The tangent is computed two
independent ways: assembled into a CSR matrix and multiplied (the sparse
baseline of Sec. 3.2.2) and as a naive cell loop (Alg. 1 of Sec. 2.4 with the
tangent tensor formed explicitly and full basis sums instead of sum
factorization).  No caching, no sum factorization, no directional-derivative
trick.

Constrained degrees of freedom are treated as identity rows and columns:
the apply reads w as zero there and returns v_c = w_c; residual entries at
constrained dofs are zero.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import material, material_split
from .mesh import BoxMesh


class Problem:
    def __init__(self, mesh: BoxMesh, mu: float, lam: float, constrained_dofs=None,
                 elem_mu_lam=None, chunk: int = 1024, model: str = "nh"):
        """model "nh": eq. hypref with (mu, lam); "split": eq. hypcomplex with
        (mu, kappa) passed in the lam slot (and in elem_mu_lam)."""
        if model not in ("nh", "split"):
            raise ValueError(f"unknown model {model}")
        self.model = model
        self.mat = material if model == "nh" else material_split
        self.mesh = mesh
        self.mu, self.lam = float(mu), float(lam)
        self.chunk = int(chunk)
        self.elem_mu_lam = None if elem_mu_lam is None else np.asarray(elem_mu_lam, np.float64).reshape(-1, 2)
        mask = np.zeros(mesh.n_dofs, dtype=bool)
        if constrained_dofs is not None and len(constrained_dofs):
            mask[np.asarray(constrained_dofs, dtype=np.int64)] = True
        self.constrained = mask

    # ------------------------------------------------------------ helpers
    def _chunks(self, elems=None):
        elems = np.arange(self.mesh.n_elems) if elems is None else np.asarray(elems)
        for s in range(0, elems.size, self.chunk):
            yield elems[s:s + self.chunk]

    def _material(self, elems):
        if self.elem_mu_lam is None:
            return self.mu, self.lam
        ml = self.elem_mu_lam[elems]
        return ml[:, 0][:, None], ml[:, 1][:, None]     # broadcast over q

    def _local(self, vec, elems):
        """vec restricted to cells: [E, 3, n3]."""
        return vec[self.mesh.elem_dofs(elems)]

    def deformation_gradient(self, u, elems=None):
        """F[e, q, i, A] = d_iA + sum_a u_(a,i) Grad_A N_a at every quadrature point."""
        gradN, _ = self.mesh.geometry(elems)
        ue = self._local(u, np.arange(self.mesh.n_elems) if elems is None else elems)
        return np.eye(3) + np.einsum("eia,eqaA->eqiA", ue, gradN)

    def min_jacobian(self, u) -> float:
        m = np.inf
        for el in self._chunks():
            F = self.deformation_gradient(u, el)
            m = min(m, float(np.min(np.linalg.det(F).real)))
        return m

    # ------------------------------------------------------------ energy / residual
    def energy(self, u):
        total = 0.0
        for el in self._chunks():
            gradN, JxW = self.mesh.geometry(el)
            F = np.eye(3) + np.einsum("eia,eqaA->eqiA", self._local(u, el), gradN)
            mu, lam = self._material(el)
            total = total + np.sum(JxW * self.mat.energy_density(F, mu, lam))
        return total

    def residual(self, u):
        R = np.zeros(self.mesh.n_dofs, dtype=np.result_type(u, np.float64))
        for el in self._chunks():
            gradN, JxW = self.mesh.geometry(el)
            F = np.eye(3) + np.einsum("eia,eqaA->eqiA", self._local(u, el), gradN)
            mu, lam = self._material(el)
            P = self.mat.piola(F, mu, lam)
            Re = np.einsum("eq,eqiA,eqaA->eia", JxW, P, gradN)
            np.add.at(R, self.mesh.elem_dofs(el).ravel(), Re.ravel())
        R[self.constrained] = 0.0
        return R

    # ------------------------------------------------------------ tangent
    def apply_naive(self, u, w, elems=None):
        """Cell loop of the tangent action over ``elems`` (all cells by default).

        Returns the full-length vector; with a subset of cells only their
        contributions are summed (used for bounded timing samples)."""
        w0 = np.where(self.constrained, 0.0, w)
        v = np.zeros(self.mesh.n_dofs, dtype=np.result_type(u, w, np.float64))
        for el in self._chunks(elems):
            gradN, JxW = self.mesh.geometry(el)
            F = np.eye(3) + np.einsum("eia,eqaA->eqiA", self._local(u, el), gradN)
            mu, lam = self._material(el)
            L = self.mat.tangent(F, mu, lam)                                  # [E,q,3,3,3,3]
            H = np.einsum("eja,eqaB->eqjB", self._local(w0, el), gradN)      # Grad w
            G = np.einsum("eqiAjB,eqjB->eqiA", L, H)                          # L : Grad w
            ve = np.einsum("eq,eqiA,eqaA->eia", JxW, G, gradN)
            np.add.at(v, self.mesh.elem_dofs(el).ravel(), ve.ravel())
        if elems is None:
            v[self.constrained] = w[self.constrained]
        return v

    def apply_at(self, u, w, dofs):
        """Exact tangent action at the selected global dofs only (sums the
        contributions of every cell touching their nodes)."""
        dofs = np.asarray(dofs, dtype=np.int64)
        cells = self.mesh.elements_of_nodes(np.unique(dofs // 3))
        v = self.apply_naive(u, w, elems=cells)
        out = v[dofs]
        c = self.constrained[dofs]
        out[c] = w[dofs[c]]
        return out

    def element_matrices(self, u, elems=None):
        """K_e[e, i, a, j, b] = sum_q JxW grad_A N_a L_iAjB grad_B N_b."""
        gradN, JxW = self.mesh.geometry(elems)
        el = np.arange(self.mesh.n_elems) if elems is None else np.asarray(elems)
        F = np.eye(3) + np.einsum("eia,eqaA->eqiA", self._local(u, el), gradN)
        mu, lam = self._material(el)
        L = self.mat.tangent(F, mu, lam)
        return np.einsum("eq,eqaA,eqiAjB,eqbB->eiajb", JxW, gradN, L, gradN, optimize=True)

    def assemble_tangent(self, u) -> sp.csr_matrix:
        """Global sparse tangent (identity rows/columns at constrained dofs)."""
        rows, cols, vals = [], [], []
        n3 = self.mesh.n3
        for el in self._chunks():
            Ke = self.element_matrices(u, el)                              # [E,3,n3,3,n3]
            d = self.mesh.elem_dofs(el).reshape(len(el), 3 * n3)           # (i, a) order
            rows.append(np.repeat(d, 3 * n3, axis=1).ravel())
            cols.append(np.tile(d, (1, 3 * n3)).ravel())
            vals.append(Ke.reshape(len(el), -1))
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        vals = np.concatenate([v.ravel() for v in vals])
        c = self.constrained
        keep = ~(c[rows] | c[cols])
        n = self.mesh.n_dofs
        K = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n)).tocsr()
        if c.any():
            K = K + sp.diags(c.astype(np.float64), format="csr")
        K.sum_duplicates()
        return K
