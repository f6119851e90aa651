"""1D quadrature and shape functions of the tensor-product Q_p element.

The paper discretises with Q_p hexahedra (Sec. 2.2) and integrates with
(p+1)^d quadrature points per cell (Sec. 2.4; Table 2 pairs q = p+1 with p).
It does not name the support points of the Lagrange basis; this oracle uses
Gauss-Lobatto-Legendre points (equispaced for p <= 2) and Gauss-Legendre
quadrature, both mapped to the unit interval [0, 1].
"""

from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_rule(nq: int):
    """Gauss-Legendre points and weights on [0, 1] (exact for degree 2*nq-1).

    Library routine (numpy's Golub-Welsch based ``leggauss``) on [-1, 1],
    affinely mapped to [0, 1].
    """
    x, w = npleg.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def gll_points(p: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre points of degree p on [0, 1]: the end points and
    the roots of the derivative of the Legendre polynomial P_p."""
    if p < 1:
        raise ValueError("degree must be >= 1")
    if p == 1:
        return np.array([0.0, 1.0])
    interior = npleg.Legendre.basis(p).deriv().roots().real
    pts = np.concatenate([[-1.0], np.sort(interior), [1.0]])
    return 0.5 * (pts + 1.0)


def lagrange_values(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """``L[i, k] = l_i(x_k)`` for the Lagrange polynomials through ``nodes``.

    Plain product formula l_i(x) = prod_{j != i} (x - x_j) / (x_i - x_j).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x)
    n = nodes.size
    out = np.ones((n, x.size), dtype=np.result_type(x, np.float64))
    for i in range(n):
        for j in range(n):
            if j != i:
                out[i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return out


def lagrange_derivatives(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """``D[i, k] = l_i'(x_k)`` by the product rule:
    l_i'(x) = sum_{m != i} 1/(x_i - x_m) prod_{j != i, m} (x - x_j)/(x_i - x_j)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x)
    n = nodes.size
    out = np.zeros((n, x.size), dtype=np.result_type(x, np.float64))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(x.shape, 1.0 / (nodes[i] - nodes[m]), dtype=out.dtype)
            for j in range(n):
                if j != i and j != m:
                    term = term * (x - nodes[j]) / (nodes[i] - nodes[j])
            out[i] += term
    return out


class TensorBasis:
    """Full (not sum-factorised) 3D basis of Q_p at the (p+1)^3 Gauss points.

    Node ``a = i + n*(j + n*k)`` is the product l_i(xi_0) l_j(xi_1) l_k(xi_2);
    quadrature point ``q = qx + nq*(qy + nq*qz)`` likewise.
    Attributes
    ----------
    values : [nq3, n3]      N_a(xi_q)
    grads  : [nq3, n3, 3]   dN_a/dxi_A (xi_q)
    weights: [nq3]          tensor Gauss weights on the unit cube
    points : [nq3, 3]       reference coordinates of the quadrature points
    """

    def __init__(self, degree: int, nq: int | None = None):
        p = int(degree)
        nq = p + 1 if nq is None else int(nq)
        self.degree, self.n, self.nq = p, p + 1, nq
        self.nodes_1d = gll_points(p)
        self.qpts_1d, self.qwts_1d = gauss_rule(nq)
        L = lagrange_values(self.nodes_1d, self.qpts_1d)        # [n, nq]
        dL = lagrange_derivatives(self.nodes_1d, self.qpts_1d)  # [n, nq]
        n = self.n
        n3, nq3 = n ** 3, nq ** 3
        values = np.zeros((nq3, n3))
        grads = np.zeros((nq3, n3, 3))
        weights = np.zeros(nq3)
        points = np.zeros((nq3, 3))
        for qz in range(nq):
            for qy in range(nq):
                for qx in range(nq):
                    q = qx + nq * (qy + nq * qz)
                    weights[q] = self.qwts_1d[qx] * self.qwts_1d[qy] * self.qwts_1d[qz]
                    points[q] = (self.qpts_1d[qx], self.qpts_1d[qy], self.qpts_1d[qz])
                    for k in range(n):
                        for j in range(n):
                            for i in range(n):
                                a = i + n * (j + n * k)
                                values[q, a] = L[i, qx] * L[j, qy] * L[k, qz]
                                grads[q, a, 0] = dL[i, qx] * L[j, qy] * L[k, qz]
                                grads[q, a, 1] = L[i, qx] * dL[j, qy] * L[k, qz]
                                grads[q, a, 2] = L[i, qx] * L[j, qy] * dL[k, qz]
        self.values, self.grads, self.weights, self.points = values, grads, weights, points
