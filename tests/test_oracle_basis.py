"""Pins of the oracle's 1D/3D basis and quadrature against closed forms."""

import numpy as np
import pytest

from oracle import basis


@pytest.mark.parametrize("nq", [1, 2, 3, 4, 5, 7, 8])
def test_gauss_rule_exact_to_degree_2nq_minus_1(nq):
    x, w = basis.gauss_rule(nq)
    for k in range(2 * nq):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-14
    # and not exact one degree higher (so it is the nq-point Gauss rule, not more)
    assert abs(np.sum(w * x ** (2 * nq)) - 1.0 / (2 * nq + 1)) > 1e-12


def test_gll_points_closed_forms():
    s = lambda t: 0.5 * (np.asarray(t) + 1.0)
    assert np.allclose(basis.gll_points(1), [0.0, 1.0], atol=1e-15)
    assert np.allclose(basis.gll_points(2), [0.0, 0.5, 1.0], atol=1e-15)
    r5 = 1.0 / np.sqrt(5.0)
    assert np.allclose(basis.gll_points(3), s([-1, -r5, r5, 1]), atol=1e-15)
    r37 = np.sqrt(3.0 / 7.0)
    assert np.allclose(basis.gll_points(4), s([-1, -r37, 0, r37, 1]), atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_lagrange_cardinal_partition_and_reproduction(p):
    nodes = basis.gll_points(p)
    L = basis.lagrange_values(nodes, nodes)
    assert np.allclose(L, np.eye(p + 1), atol=1e-13)
    x = np.linspace(-0.1, 1.1, 17)
    V = basis.lagrange_values(nodes, x)
    D = basis.lagrange_derivatives(nodes, x)
    assert np.allclose(V.sum(axis=0), 1.0, atol=1e-12)
    assert np.allclose(D.sum(axis=0), 0.0, atol=1e-10)
    rng = np.random.default_rng(p)
    c = rng.standard_normal(p + 1)
    poly = np.polynomial.Polynomial(c)
    assert np.allclose(poly(nodes) @ V, poly(x), atol=1e-11)
    assert np.allclose(poly(nodes) @ D, poly.deriv()(x), atol=1e-9)


@pytest.mark.parametrize("p", [1, 2, 4])
def test_tensor_basis(p):
    tb = basis.TensorBasis(p)
    assert np.allclose(tb.values.sum(axis=1), 1.0, atol=1e-13)
    assert np.allclose(tb.grads.sum(axis=1), 0.0, atol=1e-11)
    assert abs(tb.weights.sum() - 1.0) < 1e-14
    # integrate x^a y^b z^c exactly for a, b, c <= 2q-1
    X = tb.points
    for (a, b, c) in [(0, 0, 0), (1, 2, 0), (2 * p + 1, 0, 1), (p, p, p)]:
        exact = 1.0 / ((a + 1) * (b + 1) * (c + 1))
        assert abs(np.sum(tb.weights * X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** c) - exact) < 1e-14
    # numbering: node a = i + n(j + n k), point q = qx + nq(qy + nq qz)
    n, nq = p + 1, tb.nq
    Lx = basis.lagrange_values(tb.nodes_1d, tb.qpts_1d)
    i, j, k = 1 % n, 0, n - 1
    qx, qy, qz = 1 % nq, 0, nq - 1
    a = i + n * (j + n * k)
    q = qx + nq * (qy + nq * qz)
    assert abs(tb.values[q, a] - Lx[i, qx] * Lx[j, qy] * Lx[k, qz]) < 1e-15
