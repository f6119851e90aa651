"""Pins of the split neo-Hookean oracle (eq. hypcomplex): P and L against
complex-step derivatives of Psi and P, symmetry, the u = 0 limit against
textbook linear elasticity with Lame constants (kappa - 2 mu / 3, mu),
isochoric invariance of the deviatoric part, and K.w of the assembled
tangent against the complex step of the residual."""

import numpy as np
import pytest

import synthetic
from oracle import linelast, material_split as ms
from oracle.fem import Problem
from oracle.mesh import BoxMesh

H = 1e-30


def _F(seed, n=6, amp=0.25):
    rng = np.random.default_rng(seed)
    return np.eye(3) + amp * rng.normal(size=(n, 3, 3))


def test_piola_is_derivative_of_energy():
    F = _F(1)
    mu, kappa = 1.3, 7.0
    P = ms.piola(F, mu, kappa)
    rng = np.random.default_rng(2)
    for _ in range(5):
        W = rng.normal(size=(3, 3))
        cs = ms.energy_density(F + 1j * H * W, mu, kappa).imag / H
        np.testing.assert_allclose(cs, np.einsum("nij,ij->n", P, W), rtol=1e-13, atol=1e-14)


def test_tangent_is_derivative_of_piola_and_major_symmetric():
    F = _F(3)
    mu, kappa = 0.7, 20.0
    L = ms.tangent(F, mu, kappa)
    for j in range(3):
        for B in range(3):
            E = np.zeros((3, 3))
            E[j, B] = 1.0
            cs = ms.piola(F + 1j * H * E, mu, kappa).imag / H
            np.testing.assert_allclose(L[:, :, :, j, B], cs, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(L, np.einsum("niAjB->njBiA", L), rtol=1e-12, atol=1e-12)


def test_reference_state_and_volume_preserving_invariance():
    mu, kappa = 1.0, 5.0
    np.testing.assert_allclose(ms.piola(np.eye(3)[None], mu, kappa), 0.0, atol=1e-15)
    assert abs(ms.energy_density(np.eye(3)[None], mu, kappa)[0]) < 1e-15
    # a pure dilation has no isochoric energy
    F = 1.1 * np.eye(3)[None]
    J = 1.1 ** 3
    np.testing.assert_allclose(ms.energy_density(F, mu, kappa), 0.5 * kappa * (0.5 * (J * J - 1) - np.log(J)),
                               rtol=1e-14)


def test_small_strain_limit_is_linear_elasticity():
    mesh = BoxMesh(2, 2, 2, 2, synthetic.box_vertices(2, 2, 2))
    mu, kappa = 1.0, 9.0
    P = Problem(mesh, mu, kappa, model="split")
    K = P.assemble_tangent(np.zeros(mesh.n_dofs)).toarray()
    Klin = linelast.assemble(mesh, kappa - 2.0 * mu / 3.0, mu).toarray()
    np.testing.assert_allclose(K, Klin, rtol=1e-12, atol=1e-12 * np.abs(Klin).max())


@pytest.mark.parametrize("degree", [1, 2])
def test_apply_is_complex_step_of_residual(degree):
    nx = 2
    verts = synthetic.box_vertices(nx, nx, nx, (1.0, 1.0, 1.0), 0.1, np.random.default_rng(4))
    mesh = BoxMesh(nx, nx, nx, degree, verts)
    P = Problem(mesh, 1.0, 12.0, model="split")
    u = synthetic.sine_displacement(nx, nx, nx, degree, 0.05, np.random.default_rng(5))
    w = np.random.default_rng(6).normal(size=mesh.n_dofs)
    cs = P.residual(u + 1j * H * w).imag / H
    np.testing.assert_allclose(P.apply_naive(u, w), cs, rtol=1e-11, atol=1e-11 * np.abs(cs).max())
    np.testing.assert_allclose(P.assemble_tangent(u) @ w, cs, rtol=1e-11, atol=1e-11 * np.abs(cs).max())
    r = P.residual(u)
    E = lambda v: P.energy(v)
    np.testing.assert_allclose(E(u + 1j * H * w).imag / H, r @ w, rtol=1e-12)
