"""Pins of the oracle's general hexahedral mesh (canonical Q_p numbering).

The numbering is pinned geometrically: every cell's trilinear image of its
support points must land on the global node it is numbered to (shared nodes
coincide) and distinct global nodes must be distinct points, so the
numbering is a bijection between support points and ids; it is exercised
with random vertex relabelling and random rotations of every cell's local
order, at degrees where edges and faces carry several nodes.  The operator
on a general mesh is pinned against the structured box (itself pinned by
complex step, brute force and closed forms), through the permutation that
matches node positions, and by the complex step and the patch test on an
unstructured mesh."""

import numpy as np
import pytest
from scipy.spatial import cKDTree

import synthetic
from oracle import material
from oracle.fem import Problem
from oracle.mesh import BoxMesh, HexMesh

H_CS = 1e-30


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _unstructured(m=1, seed=3, relabel=True):
    v, c = synthetic.cube_in_cube(m, jitter=0.1, rng=np.random.default_rng(seed))
    if relabel:
        v, c, _, _ = synthetic.relabel(v, c, np.random.default_rng(seed + 1), shuffle_cells=True)
    return v, c


def node_map(pos_a, pos_b):
    """perm with pos_b[perm[i]] == pos_a[i] (asserting a bijection)."""
    d, perm = cKDTree(pos_b).query(pos_a)
    assert d.max() < 1e-12
    assert np.unique(perm).size == perm.size
    return perm


def dof_map(perm):
    return (3 * perm[:, None] + np.arange(3)).reshape(-1)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_numbering_is_a_bijection_of_support_points(p):
    v, c = _unstructured()
    H = HexMesh(v, c, p)
    cp = H.cell_node_positions()
    pos = H.node_positions()
    # every (cell, local node) lands on its global node ...
    assert np.abs(cp - pos[H.elem_nodes]).max() < 1e-14
    # ... and distinct ids are distinct points
    d, _ = cKDTree(pos).query(pos, k=2)
    assert d[:, 1].min() > 1e-6
    # every id is used
    assert np.unique(H.elem_nodes).size == H.n_nodes


def test_numbering_layout():
    v, c = _unstructured(relabel=False)
    p = 3
    H = HexMesh(v, c, p)
    nv = v.shape[0]
    # vertices first, then (p-1) nodes per edge, (p-1)^2 per face, (p-1)^3 per cell
    assert H.n_nodes == nv + 2 * H.n_edges + 4 * H.n_faces + 8 * H.n_elems
    for e in range(H.n_elems):
        corners = H.elem_nodes[e][[0, 3, 12, 15, 48, 51, 60, 63]]
        assert np.array_equal(corners, c[e])
    # the edge nodes of the lowest edge come right after the vertices, from its lower end
    pos = H.node_positions()
    lo, hi = sorted({(min(row[a], row[b]), max(row[a], row[b]))
                     for row in c.tolist() for a, b in [(0, 1), (0, 2), (0, 4), (1, 3), (1, 5), (2, 3),
                                                         (2, 6), (3, 7), (4, 5), (4, 6), (5, 7), (6, 7)]})[0]
    t = H.basis.nodes_1d
    for s in (1, 2):
        assert np.allclose(pos[nv + s - 1], (1 - t[s]) * v[lo] + t[s] * v[hi], atol=1e-14)


def test_box_node_count():
    for p in (1, 2, 3):
        v = synthetic.box_vertices(3, 2, 4)
        H = HexMesh(v, synthetic.box_cells(3, 2, 4), p)
        assert H.n_nodes == (3 * p + 1) * (2 * p + 1) * (4 * p + 1)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_operator_matches_structured_box(p):
    nx, ny, nz = 3, 2, 2
    rng = np.random.default_rng(21)
    v = synthetic.box_vertices(nx, ny, nz, (1.0, 0.8, 1.2), 0.12, rng)
    B = BoxMesh(nx, ny, nz, p, v)
    v2, c2, _, _ = synthetic.relabel(v, synthetic.box_cells(nx, ny, nz), np.random.default_rng(22),
                                     shuffle_cells=True)
    H = HexMesh(v2, c2, p)
    perm = node_map(H.node_positions(), B.node_positions())    # hex node i = box node perm[i]
    dm = dof_map(perm)
    u_b = synthetic.sine_displacement(nx, ny, nz, p, 0.05, np.random.default_rng(23))
    w_b = np.random.default_rng(24).standard_normal(B.n_dofs)
    PB, PH = Problem(B, 1.0, 10.0), Problem(H, 1.0, 10.0)
    assert _rel(PH.apply_naive(u_b[dm], w_b[dm]), PB.apply_naive(u_b, w_b)[dm]) < 1e-13
    assert _rel(PH.residual(u_b[dm]), PB.residual(u_b)[dm]) < 1e-13
    assert abs(PH.energy(u_b[dm]) - PB.energy(u_b)) < 1e-13 * abs(PB.energy(u_b))


@pytest.mark.parametrize("p", [2, 3])
def test_tangent_is_complex_step_of_residual_unstructured(p):
    v, c = _unstructured()
    H = HexMesh(v, c, p)
    P = Problem(H, 1.0, 10.0)
    u = synthetic.sine_field(H.node_positions(), 0.04, np.random.default_rng(31))
    w = np.random.default_rng(32).standard_normal(H.n_dofs)
    cs = P.residual(u + 1j * H_CS * w).imag / H_CS
    assert _rel(P.apply_naive(u, w), cs) < 1e-13
    assert _rel(P.assemble_tangent(u) @ w, cs) < 1e-13


def test_patch_test_unstructured():
    v, c = _unstructured()
    H = HexMesh(v, c, 2)
    P = Problem(H, 1.0, 10.0)
    X = H.node_positions()
    Hm = np.array([[0.05, 0.02, -0.03], [0.01, -0.04, 0.02], [0.03, 0.01, 0.06]])
    u = (X @ Hm.T).reshape(-1)
    F = np.eye(3) + Hm
    E = P.energy(u)
    assert abs(E - material.energy_density(F[None], 1.0, 10.0)[0]) < 1e-13 * abs(E)
    R = P.residual(u).reshape(-1, 3)
    on_bnd = np.any((np.abs(X) < 1e-12) | (np.abs(X - 1.0) < 1e-12), axis=1)
    assert np.abs(R[~on_bnd]).max() < 1e-12 * np.abs(R).max()


def test_rotating_cells_only_permutes_interior_nodes():
    v, c = _unstructured(relabel=False)
    v2, c2, _, _ = synthetic.relabel(v, c, np.random.default_rng(41), shuffle_vertices=False)
    A, B = HexMesh(v, c, 3), HexMesh(v2, c2, 3)
    n_shared = v.shape[0] + 2 * A.n_edges + 4 * A.n_faces
    perm = node_map(B.node_positions(), A.node_positions())
    assert np.array_equal(perm[:n_shared], np.arange(n_shared))


def test_invalid_meshes_are_rejected():
    v, c = _unstructured(relabel=False)
    bad = c.copy()
    bad[0, 0] = v.shape[0]
    with pytest.raises(ValueError):
        HexMesh(v, bad, 2)
    bad = c.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(ValueError):
        HexMesh(v, bad, 2)
    # two cells on the same 4 face vertices but with crossed edges
    v2 = synthetic.box_vertices(2, 1, 1)
    c2 = synthetic.box_cells(2, 1, 1).astype(np.int64)
    x = c2[1].copy()
    c2[1, [0, 2]] = x[[2, 0]]
    with pytest.raises(ValueError):
        HexMesh(v2, c2, 2)
    # an inverted cell is refused by the geometry
    c3 = synthetic.box_cells(2, 1, 1).astype(np.int64)
    c3[0] = c3[0][[1, 0, 3, 2, 5, 4, 7, 6]]
    with pytest.raises(ValueError):
        HexMesh(v2, c3, 1).geometry()
