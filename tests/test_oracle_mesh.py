"""Pins of the oracle's geometry: volumes, affine maps, exact gradients of
linear fields, connectivity."""

import numpy as np
import pytest

import synthetic
from oracle.mesh import BoxMesh


def _mesh(nx, ny, nz, p, lengths=(1, 1, 1), jitter=0.0, seed=5):
    rng = np.random.default_rng(seed)
    v = synthetic.box_vertices(nx, ny, nz, lengths, jitter, rng if jitter else None)
    return BoxMesh(nx, ny, nz, p, v)


@pytest.mark.parametrize("p,jit", [(1, 0.0), (2, 0.1), (3, 0.1), (2, 0.0)])
def test_volume(p, jit):
    m = _mesh(3, 2, 4, p, lengths=(2.0, 1.0, 0.5), jitter=jit)
    _, JxW = m.geometry()
    assert abs(JxW.sum() - 1.0) < 1e-13


def test_affine_vertices_give_constant_jacobian():
    m = _mesh(2, 3, 2, 2, lengths=(1.0, 1.0, 1.0))
    A = np.array([[1.2, 0.3, -0.1], [0.05, 0.9, 0.2], [0.1, -0.2, 1.1]])
    b = np.array([0.3, -1.0, 2.0])
    m2 = BoxMesh(2, 3, 2, 2, m.vertices @ A.T + b)
    Jg = m2.jacobians()
    h = np.diag([1 / 2, 1 / 3, 1 / 2])
    assert np.allclose(Jg, (A @ h)[None, None], atol=1e-14)
    _, JxW = m2.geometry()
    assert abs(JxW.sum() - np.linalg.det(A)) < 1e-13


def test_node_positions_regular_grid():
    m = _mesh(2, 2, 3, 2)
    pos = m.node_positions()
    Nx, Ny, Nz = m.nodes_per_dir
    K, J, I = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    ref = np.stack([I.ravel() / (Nx - 1), J.ravel() / (Ny - 1), K.ravel() / (Nz - 1)], axis=1)
    assert np.allclose(pos, ref, atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gradient_of_interpolated_linear_field_is_exact(p):
    m = _mesh(2, 3, 2, p, jitter=0.15)
    pos = m.node_positions()
    c = np.array([0.7, -1.3, 2.1])
    f = pos @ c + 0.4
    gradN, _ = m.geometry()
    fe = f[m.elem_nodes]                                   # [E, n3]
    g = np.einsum("ea,eqaA->eqA", fe, gradN)
    assert np.allclose(g, c[None, None], atol=1e-12)


def test_elements_of_nodes_brute_force():
    m = _mesh(3, 2, 2, 2)
    rng = np.random.default_rng(0)
    for node in rng.integers(0, m.n_nodes, 20):
        brute = np.where((m.elem_nodes == node).any(axis=1))[0]
        assert np.array_equal(m.elements_of_nodes([node]), brute)


def test_connectivity_numbering():
    m = _mesh(2, 2, 2, 2)
    # cell 0 local node (i,j,k)=(2,1,0) is node (2,1,0) = 2 + 5*1
    assert m.elem_nodes[0, 2 + 3 * 1] == 2 + 5 * 1
    # cell (1,1,1) = 7, local (0,0,0) = node (2,2,2)
    assert m.elem_nodes[7, 0] == 2 + 5 * (2 + 5 * 2)
    assert m.n_dofs == 3 * 125
