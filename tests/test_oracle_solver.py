"""The oracle's Newton driver: converged residual, exact Dirichlet values,
and path independence of the hyperelastic solution."""

import numpy as np

import synthetic
import oracle
from oracle.fem import Problem
from oracle.mesh import BoxMesh


def _beam(lam=100.0):
    nx, ny, nz, L = 6, 2, 2, (3.0, 1.0, 1.0)
    mesh = BoxMesh(nx, ny, nz, 2, synthetic.box_vertices(nx, ny, nz, L))
    cdofs, _ = synthetic.clamp_and_twist(nx, ny, nz, 2, L, 0.0)
    return (nx, ny, nz, L), mesh, Problem(mesh, 1.0, lam, constrained_dofs=cdofs)


def test_newton_converges_with_exact_boundary_values():
    (nx, ny, nz, L), mesh, P = _beam()
    d, v = synthetic.clamp_and_twist(nx, ny, nz, 2, L, np.deg2rad(10.0))
    u, hist = oracle.solver.newton(P, np.zeros(mesh.n_dofs), d, v, atol=1e-10)
    assert hist[-1] <= 1e-10 and np.array_equal(u[d], v)
    assert np.linalg.norm(P.residual(u)) <= 1e-10
    assert P.min_jacobian(u) > 0.5
    # quadratic convergence at the end
    assert hist[-1] <= max(1e3 * hist[-2] ** 2, 1e-12)


def test_solution_is_path_independent():
    (nx, ny, nz, L), mesh, P = _beam()
    u1 = np.zeros(mesh.n_dofs)
    for k in (1, 2):
        d, v = synthetic.clamp_and_twist(nx, ny, nz, 2, L, np.deg2rad(6.0 * k))
        u1, _ = oracle.solver.newton(P, u1, d, v, atol=1e-11)
    d, v = synthetic.clamp_and_twist(nx, ny, nz, 2, L, np.deg2rad(12.0))
    u2, _ = oracle.solver.newton(P, np.zeros(mesh.n_dofs), d, v, atol=1e-11)
    assert np.linalg.norm(u1 - u2) <= 1e-9 * np.linalg.norm(u2)


def test_twist_data_is_a_rigid_rotation_of_the_end_face():
    nx, ny, nz, L = 4, 2, 2, (2.0, 1.0, 1.0)
    th = 0.3
    d, v = synthetic.clamp_and_twist(nx, ny, nz, 2, L, th)
    mesh = BoxMesh(nx, ny, nz, 2, synthetic.box_vertices(nx, ny, nz, L))
    X = mesh.node_positions()
    u = np.zeros(mesh.n_dofs)
    u[d] = v
    U = u.reshape(-1, 3)
    right = np.isclose(X[:, 0], L[0])
    left = np.isclose(X[:, 0], 0.0)
    assert np.all(U[left] == 0.0)
    # distances between end-face points are preserved and the axis point is fixed
    x = X[right] + U[right]
    c = np.array([L[0], 0.5, 0.5])
    assert np.allclose(np.linalg.norm(x - c, axis=1), np.linalg.norm(X[right] - c, axis=1), atol=1e-14)
    ang = np.arctan2(x[:, 2] - 0.5, x[:, 1] - 0.5) - np.arctan2(X[right][:, 2] - 0.5, X[right][:, 1] - 0.5)
    r = np.linalg.norm(X[right][:, 1:] - 0.5, axis=1) > 1e-12
    assert np.allclose(np.mod(ang[r] + np.pi, 2 * np.pi) - np.pi, th, atol=1e-13)
