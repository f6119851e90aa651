"""Pins of the oracle's discrete residual and tangent.

None of these compares the oracle with itself: every check is a derivative
computed another way (complex step, central differences, dense brute force),
an invariant (symmetry, rigid modes, objectivity), a closed form (patch test)
or an independent textbook assembly (small-strain limit)."""

import numpy as np
import pytest

import synthetic
from oracle import linelast
from oracle.fem import Problem
from oracle.mesh import BoxMesh

H_CS = 1e-30


def _problem(name="cube4_q2_jit", constrained=None):
    cfg = synthetic.get_config(name)
    mesh = BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, cfg.vertices())
    return cfg, Problem(mesh, cfg.mu, cfg.lam, constrained_dofs=constrained)


def _small(p, nx=2, ny=2, nz=2, jitter=0.12, amp=0.03, seed=11, lam=10.0, mu=1.0):
    rng = np.random.default_rng(seed)
    v = synthetic.box_vertices(nx, ny, nz, (1.0, 1.3, 0.8), jitter, rng)
    mesh = BoxMesh(nx, ny, nz, p, v)
    u = synthetic.sine_displacement(nx, ny, nz, p, amp, np.random.default_rng(seed + 1))
    return Problem(mesh, mu, lam), u, np.random.default_rng(seed + 2)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("name", ["cube4_q2", "cube4_q2_jit"])
def test_tangent_is_complex_step_of_residual(name):
    cfg, P = _problem(name)
    u = cfg.displacement()
    K = P.assemble_tangent(u)
    for w in cfg.test_vectors()[:4]:
        cs = P.residual(u + 1j * H_CS * w).imag / H_CS
        assert _rel(K @ w, cs) < 1e-13


@pytest.mark.parametrize("p", [1, 3, 4])
def test_tangent_is_complex_step_of_residual_other_degrees(p):
    P, u, rng = _small(p)
    w = rng.standard_normal(P.mesh.n_dofs)
    cs = P.residual(u + 1j * H_CS * w).imag / H_CS
    assert _rel(P.apply_naive(u, w), cs) < 1e-13
    if p < 4:   # the p = 4 element matrices are large; the naive loop covers it
        assert _rel(P.assemble_tangent(u) @ w, cs) < 1e-13


def test_tangent_matches_central_difference_of_residual():
    cfg, P = _problem()
    u = cfg.displacement()
    w = cfg.test_vector(0)
    eps = 1e-6 * np.max(np.abs(u)) / np.max(np.abs(w))
    fd = (P.residual(u + eps * w) - P.residual(u - eps * w)) / (2 * eps)
    assert _rel(P.apply_naive(u, w), fd) < 1e-7


def test_residual_is_complex_step_of_energy():
    cfg, P = _problem()
    u = cfg.displacement()
    for w in cfg.test_vectors()[:3]:
        dE = P.energy(u + 1j * H_CS * w).imag / H_CS
        Rw = P.residual(u) @ w
        assert abs(dE - Rw) < 1e-13 * np.linalg.norm(P.residual(u)) * np.linalg.norm(w)


def test_naive_loop_equals_assembled_matrix():
    cfg, P = _problem()
    u = cfg.displacement()
    K = P.assemble_tangent(u)
    for w in cfg.test_vectors():
        assert _rel(P.apply_naive(u, w), K @ w) < 1e-14


def test_symmetry_for_eight_pairs():
    cfg, P = _problem()
    u = cfg.displacement()
    W = cfg.test_vectors()
    for k in range(8):
        w, z = W[k], W[(k + 3) % 8]
        a = w @ P.apply_naive(u, z)
        b = z @ P.apply_naive(u, w)
        assert abs(a - b) <= 1e-13 * np.linalg.norm(w) * np.linalg.norm(P.apply_naive(u, z))


def test_small_strain_limit_is_textbook_linear_elasticity():
    cfg, P = _problem()
    K0 = P.assemble_tangent(np.zeros(P.mesh.n_dofs))
    Klin = linelast.assemble(P.mesh, 2.0 * cfg.lam, cfg.mu)      # energy uses lam log^2 J
    assert abs(K0 - Klin).max() <= 1e-13 * abs(Klin).max()
    # and the nonlinear tangent departs from it linearly in the amplitude
    u = cfg.displacement()
    d1 = abs(P.assemble_tangent(1e-3 * u) - K0).max()
    d2 = abs(P.assemble_tangent(2e-3 * u) - K0).max()
    assert 1.9 < d2 / d1 < 2.1


def test_rigid_translations_in_kernel():
    cfg, P = _problem()
    u = cfg.displacement()
    scale = np.linalg.norm(P.apply_naive(u, cfg.test_vector(0)))
    for c in range(3):
        t = np.zeros(P.mesh.n_dofs)
        t[c::3] = 1.0
        assert np.linalg.norm(P.apply_naive(u, t)) <= 1e-12 * scale


def test_infinitesimal_rotations_in_kernel_at_zero_state():
    cfg, P = _problem()
    X = P.mesh.node_positions()
    zero = np.zeros(P.mesh.n_dofs)
    scale = np.linalg.norm(P.apply_naive(zero, cfg.test_vector(0)))
    for omega in np.eye(3):
        r = np.cross(omega, X).reshape(-1)
        assert np.linalg.norm(P.apply_naive(zero, r)) <= 1e-12 * scale
    # a finite state breaks it (the geometric stiffness sees the rotation)
    r = np.cross(np.array([0.0, 0.0, 1.0]), X).reshape(-1)
    assert np.linalg.norm(P.apply_naive(cfg.displacement(), r)) > 1e-6 * scale


def test_objectivity_of_residual():
    cfg, P = _problem()
    u = cfg.displacement().reshape(-1, 3)
    X = P.mesh.node_positions()
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th), 0.0], [np.sin(th), np.cos(th), 0.0], [0.0, 0.0, 1.0]])
    Q = Q @ np.array([[1, 0, 0], [0, np.cos(0.3), -np.sin(0.3)], [0, np.sin(0.3), np.cos(0.3)]])
    uQ = (X + u) @ Q.T - X
    R = P.residual(u.reshape(-1)).reshape(-1, 3)
    RQ = P.residual(uQ.reshape(-1)).reshape(-1, 3)
    assert np.abs(RQ - R @ Q.T).max() <= 1e-13 * np.abs(R).max() * 10


def test_patch_test_affine_displacement_on_jittered_mesh():
    from oracle import material
    cfg, P = _problem("cube4_q2_jit")
    X = P.mesh.node_positions()
    Hm = np.array([[0.05, 0.02, -0.03], [0.01, -0.04, 0.02], [0.03, 0.01, 0.06]])
    u = (X @ Hm.T).reshape(-1)
    F = np.eye(3) + Hm
    # energy is exactly Psi(F) * volume
    E = P.energy(u)
    assert abs(E - material.energy_density(F[None], cfg.mu, cfg.lam)[0] * 1.0) < 1e-13 * abs(E)
    # interior nodes are in equilibrium; boundary nodes carry the traction P N
    R = P.residual(u).reshape(-1, 3)
    interior = ~P.mesh.boundary_nodes()
    assert np.abs(R[interior]).max() < 1e-13 * np.abs(R).max()
    # global balance: the residuals of a homogeneous stress state sum to zero
    assert np.abs(R.sum(axis=0)).max() < 1e-13 * np.abs(R).max()


def test_patch_residual_moments():
    # x is in the discrete space (its interpolant is the trilinear geometry map), so
    # sum_a R_(a,c) x_a = int_Omega P : Grad(x e_c) dV = P_c0 * volume exactly
    from oracle import material
    cfg, P = _problem("cube4_q2_jit")
    X = P.mesh.node_positions()
    Hm = np.array([[0.04, -0.01, 0.02], [0.02, 0.03, -0.01], [-0.02, 0.01, -0.05]])
    u = (X @ Hm.T).reshape(-1)
    R = P.residual(u).reshape(-1, 3)
    F = np.eye(3) + Hm
    Pm = material.piola(F[None], cfg.mu, cfg.lam)[0]
    # test field phi = x (linear): sum_a R_a . e_c x_a = int_Omega P : Grad(x e_c) = P[c, 0] * vol
    for c in range(3):
        s = np.sum(R[:, c] * X[:, 0])
        assert abs(s - Pm[c, 0]) < 1e-13 * max(1.0, np.abs(Pm).max())


def test_dense_complex_step_jacobian_equals_assembled_matrix_small():
    P, u, _ = _small(2)
    n = P.mesh.n_dofs
    K = P.assemble_tangent(u).toarray()
    Kcs = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        Kcs[:, j] = P.residual(u + 1j * H_CS * e).imag / H_CS
    assert np.abs(K - Kcs).max() <= 1e-13 * np.abs(K).max()


@pytest.mark.slow
def test_dense_complex_step_jacobian_equals_assembled_matrix_cube4():
    cfg, P = _problem("cube4_q2")
    u = cfg.displacement()
    n = P.mesh.n_dofs
    K = P.assemble_tangent(u).toarray()
    amax = np.abs(K).max()
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        col = P.residual(u + 1j * H_CS * e).imag / H_CS
        assert np.abs(K[:, j] - col).max() <= 1e-13 * amax


def test_apply_at_sampled_dofs_matches_full_apply():
    cfg, P = _problem()
    u, w = cfg.displacement(), cfg.test_vector(0)
    v = P.apply_naive(u, w)
    dofs = np.random.default_rng(0).choice(P.mesh.n_dofs, 40, replace=False)
    assert np.allclose(P.apply_at(u, w, dofs), v[dofs], rtol=1e-13, atol=1e-13 * np.abs(v).max())


def test_constraints_identity_rows_and_columns():
    cfg, P0 = _problem()
    nodes_left = np.where(P0.mesh.node_positions()[:, 0] < 1e-12)[0]
    cdofs = (3 * nodes_left[:, None] + np.arange(3)).ravel()
    _, P = _problem(constrained=cdofs)
    u, w = cfg.displacement(), cfg.test_vector(1)
    K = P.assemble_tangent(u)
    v = P.apply_naive(u, w)
    assert _rel(v, K @ w) < 1e-14
    assert np.array_equal(v[cdofs], w[cdofs])
    # free rows ignore w at constrained dofs
    w2 = w.copy()
    w2[cdofs] = 123.0
    free = np.setdiff1d(np.arange(P.mesh.n_dofs), cdofs)
    assert np.allclose(P.apply_naive(u, w2)[free], v[free], rtol=0, atol=1e-12)
    assert abs(K - K.T).max() <= 1e-13 * abs(K).max()
    assert np.all(P.residual(u)[cdofs] == 0.0)


def test_per_cell_material_reduces_to_uniform():
    cfg, P = _problem()
    u, w = cfg.displacement(), cfg.test_vector(0)
    ml = np.tile([cfg.mu, cfg.lam], (P.mesh.n_elems, 1))
    P2 = Problem(P.mesh, 99.0, 99.0, elem_mu_lam=ml)
    assert _rel(P2.apply_naive(u, w), P.apply_naive(u, w)) < 1e-15
    # and a stiff inclusion changes the result
    ml[::7] *= 100.0
    P3 = Problem(P.mesh, 99.0, 99.0, elem_mu_lam=ml)
    assert _rel(P3.apply_naive(u, w), P.apply_naive(u, w)) > 1e-2
    cs = P3.residual(u + 1j * H_CS * w).imag / H_CS
    assert _rel(P3.apply_naive(u, w), cs) < 1e-13
