"""Split neo-Hookean material (Sec. 3.3, eq. hypcomplex): isochoric and
volumetric parts,

Psi(F) = mu/2 (tr Cbar - 3) + kappa/2 ( (J^2 - 1)/2 - log J ),
Cbar = J^{-2/3} C,  C = F^T F,  J = det F.

Derivatives written out by hand (with I1 = tr C = F:F, G = F^{-T},
a = mu J^{-2/3}, b = kappa/2 (J^2 - 1)):

P = a (F - I1/3 G) + b G

L_{iAjB} = dP_iA / dF_jB
         = -2/3 a G_jB (F_iA - I1/3 G_iA)
           + a ( d_ij d_AB - 2/3 F_jB G_iA + I1/3 G_iB G_jA )
           + kappa J^2 G_iA G_jB - b G_iB G_jA

(using dJ/dF = J G, dG_iA/dF_jB = -G_iB G_jA, dI1/dF = 2F).  The u = 0
tangent is isotropic linear elasticity with bulk modulus kappa and shear
modulus mu, i.e. Lame constants (kappa - 2 mu / 3, mu).

Same conventions as material.py: F of shape [..., 3, 3], float64 or
complex128 (the complex-step pins evaluate these functions at complex F).
TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

from __future__ import annotations

import numpy as np

I3 = np.eye(3)


def _parts(F):
    J = np.linalg.det(F)
    G = np.swapaxes(np.linalg.inv(F), -1, -2)
    I1 = np.sum(F * F, axis=(-2, -1))
    return J, G, I1


def energy_density(F, mu, kappa):
    mu = np.asarray(mu)
    kappa = np.asarray(kappa)
    J, _, I1 = _parts(F)
    return 0.5 * mu * (J ** (-2.0 / 3.0) * I1 - 3.0) + 0.5 * kappa * (0.5 * (J * J - 1.0) - np.log(J))


def piola(F, mu, kappa):
    mu = np.asarray(mu)[..., None, None]
    kappa = np.asarray(kappa)[..., None, None]
    J, G, I1 = _parts(F)
    a = mu * (J ** (-2.0 / 3.0))[..., None, None]
    b = 0.5 * kappa * (J * J - 1.0)[..., None, None]
    return a * (F - I1[..., None, None] / 3.0 * G) + b * G


def tangent(F, mu, kappa):
    mu = np.asarray(mu)[..., None, None, None, None]
    kappa = np.asarray(kappa)[..., None, None, None, None]
    J, G, I1 = _parts(F)
    a = mu * (J ** (-2.0 / 3.0))[..., None, None, None, None]
    b = 0.5 * kappa * (J * J - 1.0)[..., None, None, None, None]
    I1 = I1[..., None, None, None, None]
    J2 = (J * J)[..., None, None, None, None]
    dev = F - I1[..., 0, 0] / 3.0 * G                      # F - I1/3 G
    dd = np.einsum("ij,AB->iAjB", I3, I3)
    t_a = np.einsum("...jB,...iA->...iAjB", G, dev)        # G_jB dev_iA
    t_fg = np.einsum("...jB,...iA->...iAjB", F, G)         # F_jB G_iA
    t_gg = np.einsum("...iB,...jA->...iAjB", G, G)         # G_iB G_jA
    t_vol = np.einsum("...iA,...jB->...iAjB", G, G)        # G_iA G_jB
    return (-2.0 / 3.0 * a * t_a + a * (dd - 2.0 / 3.0 * t_fg + I1 / 3.0 * t_gg)
            + kappa * J2 * t_vol - b * t_gg)


def kirchhoff(F, mu, kappa):
    return np.einsum("...iA,...jA->...ij", piola(F, mu, kappa), F)
