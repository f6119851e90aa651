"""Pins of the oracle's material law: derivatives by complex step, symmetry,
the small-strain limit, objectivity and the current-configuration form."""

import numpy as np
import pytest

from oracle import material

MU, LAM = 1.3, 7.0
H_CS = 1e-30


def _random_F(rng, n=16, scale=0.3):
    F = np.eye(3) + scale * rng.standard_normal((n, 3, 3))
    F = F[np.linalg.det(F) > 0.2]
    return F


def test_piola_is_complex_step_derivative_of_energy():
    rng = np.random.default_rng(1)
    F = _random_F(rng)
    W = rng.standard_normal(F.shape)
    d = material.energy_density(F + 1j * H_CS * W, MU, LAM).imag / H_CS
    PW = np.sum(material.piola(F, MU, LAM) * W, axis=(-2, -1))
    assert np.max(np.abs(d - PW)) <= 1e-14 * np.max(np.abs(PW)) * 10


def test_tangent_is_complex_step_derivative_of_piola():
    rng = np.random.default_rng(2)
    F = _random_F(rng)
    W = rng.standard_normal(F.shape)
    dP = material.piola(F + 1j * H_CS * W, MU, LAM).imag / H_CS
    LW = np.einsum("niAjB,njB->niA", material.tangent(F, MU, LAM), W)
    assert np.max(np.abs(dP - LW)) <= 1e-13 * np.max(np.abs(LW))


def test_tangent_major_symmetry():
    rng = np.random.default_rng(3)
    L = material.tangent(_random_F(rng), MU, LAM)
    assert np.allclose(L, np.transpose(L, (0, 3, 4, 1, 2)), atol=1e-13)


def test_small_strain_limit_is_isotropic_linear_elasticity_with_lame_2lambda():
    # Psi = mu/2 (tr C - 3 - 2 log J) + lam log^2 J  =>  at F = I the tangent is
    # C_iAjB = lam_lin d_iA d_jB + mu (d_ij d_AB + d_iB d_Aj) with lam_lin = 2 lam.
    L = material.tangent(np.eye(3)[None], MU, LAM)[0]
    d = np.eye(3)
    ref = (2 * LAM) * np.einsum("iA,jB->iAjB", d, d) + MU * (
        np.einsum("ij,AB->iAjB", d, d) + np.einsum("iB,Aj->iAjB", d, d))
    assert np.allclose(L, ref, atol=1e-14)
    # zero stress in the reference configuration
    assert np.allclose(material.piola(np.eye(3)[None], MU, LAM), 0.0, atol=1e-15)


def test_objectivity_of_stress():
    rng = np.random.default_rng(4)
    F = _random_F(rng)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    QF = np.einsum("ij,njA->niA", Q, F)
    assert np.allclose(material.piola(QF, MU, LAM), np.einsum("ij,njA->niA", Q, material.piola(F, MU, LAM)),
                       atol=1e-13)
    assert np.allclose(material.energy_density(QF, MU, LAM), material.energy_density(F, MU, LAM), atol=1e-13)


def _psi_of_C(C, mu, lam):
    # the same energy written as a function of the right Cauchy-Green tensor
    detC = np.linalg.det(C)
    return 0.5 * mu * (np.trace(C, axis1=-2, axis2=-1) - 3.0 - np.log(detC)) + 0.25 * lam * np.log(detC) ** 2


def test_material_tangent_cc_matches_second_derivative_of_psi_of_C():
    # CC = 4 d^2 Psi/dC dC, checked by a complex step of the (symmetrised)
    # first derivative obtained by central differences of Psi(C).
    rng = np.random.default_rng(5)
    F = _random_F(rng, n=4)
    for Fk in F:
        C = Fk.T @ Fk
        CC = material.material_tangent_cc(Fk[None], MU, LAM)[0]
        A = rng.standard_normal((3, 3)); A = A + A.T
        B = rng.standard_normal((3, 3)); B = B + B.T
        # d^2 Psi [A, B] by complex step in A of a central difference in B
        e = 1e-5
        f = lambda t: _psi_of_C(C + 1j * H_CS * A + t * B, MU, LAM).imag / H_CS
        d2 = (f(e) - f(-e)) / (2 * e)
        ref = 0.25 * np.einsum("AB,ABCD,CD->", A, CC, B)
        assert abs(d2 - ref) < 1e-7 * max(1.0, abs(ref))


def test_current_configuration_form_equals_reference_form():
    # Grad du : L : Grad Du = grad du : (J c : sym(h) + h tau), h = Grad Du F^-1,
    # J c = push-forward of CC (eq. Jc).  This fixes the reading of eq. DF:cur:
    # the geometric term uses the full spatial gradient of Du on the right.
    rng = np.random.default_rng(6)
    F = _random_F(rng)
    L = material.tangent(F, MU, LAM)
    tau = material.kirchhoff(F, MU, LAM)
    Jc = material.push_forward(F, material.material_tangent_cc(F, MU, LAM))
    Finv = np.linalg.inv(F)
    for _ in range(4):
        GD = rng.standard_normal(F.shape)
        Gd = rng.standard_normal(F.shape)
        ref = np.einsum("niA,niAjB,njB->n", Gd, L, GD)
        h = np.einsum("njB,nBk->njk", GD, Finv)
        g = np.einsum("nijkl,nkl->nij", Jc, 0.5 * (h + np.swapaxes(h, 1, 2))) + np.einsum("nik,nkj->nij", h, tau)
        gd = np.einsum("niA,nAk->nik", Gd, Finv)
        cur = np.einsum("nij,nij->n", gd, g)
        assert np.allclose(cur, ref, rtol=1e-12, atol=1e-12)
        # the printed symmetric-gradient geometric term does not reproduce it
        hs = 0.5 * (h + np.swapaxes(h, 1, 2))
        g_sym = np.einsum("nijkl,nkl->nij", Jc, hs) + np.einsum("nik,nkj->nij", hs, tau)
        assert not np.allclose(np.einsum("nij,nij->n", gd, g_sym), ref, rtol=1e-6)


def test_spatial_tangent_closed_form():
    # J c = 2 lam I (x) I + 2 (mu - 2 lam log J) I^s
    rng = np.random.default_rng(7)
    F = _random_F(rng, n=6)
    Jc = material.push_forward(F, material.material_tangent_cc(F, MU, LAM))
    lJ = np.log(np.linalg.det(F))
    d = np.eye(3)
    Is = 0.5 * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d))
    ref = 2 * LAM * np.einsum("ij,kl->ijkl", d, d)[None] + 2 * (MU - 2 * LAM * lJ)[:, None, None, None, None] * Is[None]
    assert np.allclose(Jc, ref, atol=1e-12)
    # tau = mu (b - I) + 2 lam log J I
    b = np.einsum("niA,njA->nij", F, F)
    assert np.allclose(material.kirchhoff(F, MU, LAM), MU * (b - d) + 2 * LAM * lJ[:, None, None] * d, atol=1e-13)
