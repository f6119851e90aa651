"""Compressible neo-Hookean material of Sec. 3.2 (eq. hypref).

Psi(F) = mu/2 (tr C - tr I - 2 log J) + lambda (log J)^2,   C = F^T F, J = det F.

The energy is used exactly as printed: the volumetric term is lambda log^2 J
(not lambda/2 log^2 J).  Consequently the u = 0 tangent is isotropic linear
elasticity with Lame constants (2*lambda, mu).

Derivatives (Sec. 2.1, definitions of P and of the tangent tensor L):

P = dPsi/dF = mu F + (2 lambda log J - mu) F^{-T}

L_{iAjB} = d P_{iA} / d F_{jB}
         = mu d_ij d_AB + 2 lambda Finv_{Ai} Finv_{Bj}
           + (mu - 2 lambda log J) Finv_{Aj} Finv_{Bi}

Current-configuration quantities (Sec. 2.1, eqs. F:cur, DF:cur, Jc):
tau = P F^T (Kirchhoff stress) and the push-forward J c = chi(CC) of
CC = 4 d^2 Psi / dC dC.

All functions take F of shape [..., 3, 3] (float64 or complex128) and keep the
input's dtype, so they also serve the complex-step pins.
"""

from __future__ import annotations

import numpy as np

I3 = np.eye(3)


def _logdet(F):
    J = np.linalg.det(F)
    return J, np.log(J)


def energy_density(F, mu, lam):
    """Psi(F), shape F.shape[:-2]."""
    mu = np.asarray(mu)
    lam = np.asarray(lam)
    J, lJ = _logdet(F)
    trC = np.sum(F * F, axis=(-2, -1))
    return 0.5 * mu * (trC - 3.0 - 2.0 * lJ) + lam * lJ * lJ


def piola(F, mu, lam):
    """First Piola-Kirchhoff stress P = mu F + (2 lam log J - mu) F^{-T}."""
    mu = np.asarray(mu)[..., None, None]
    lam = np.asarray(lam)[..., None, None]
    J, lJ = _logdet(F)
    FinvT = np.swapaxes(np.linalg.inv(F), -1, -2)
    return mu * F + (2.0 * lam * lJ[..., None, None] - mu) * FinvT


def tangent(F, mu, lam):
    """Explicit tangent tensor L[..., i, A, j, B] = dP_iA / dF_jB (81 entries)."""
    mu = np.asarray(mu)[..., None, None, None, None]
    lam = np.asarray(lam)[..., None, None, None, None]
    J, lJ = _logdet(F)
    Finv = np.linalg.inv(F)                       # Finv[..., A, i]
    FinvT = np.swapaxes(Finv, -1, -2)             # FinvT[..., i, A] = Finv[A, i]
    dd = np.einsum("ij,AB->iAjB", I3, I3)
    t1 = np.einsum("...iA,...jB->...iAjB", FinvT, FinvT)      # Finv_Ai Finv_Bj
    t2 = np.einsum("...jA,...iB->...iAjB", FinvT, FinvT)      # Finv_Aj Finv_Bi
    return mu * dd + 2.0 * lam * t1 + (mu - 2.0 * lam * lJ[..., None, None, None, None]) * t2


def kirchhoff(F, mu, lam):
    """tau = P F^T."""
    return np.einsum("...iA,...jA->...ij", piola(F, mu, lam), F)


def material_tangent_cc(F, mu, lam):
    """CC = 4 d^2 Psi / dC dC for Psi written as a function of C:
    CC = 2 lam Cinv (x) Cinv + 2 (mu - 2 lam log J) I_{Cinv},
    (I_{Cinv})_{ABCD} = (Cinv_AC Cinv_BD + Cinv_AD Cinv_BC) / 2."""
    mu = np.asarray(mu)[..., None, None, None, None]
    lam = np.asarray(lam)[..., None, None, None, None]
    J, lJ = _logdet(F)
    C = np.einsum("...iA,...iB->...AB", F, F)
    Ci = np.linalg.inv(C)
    outer = np.einsum("...AB,...CD->...ABCD", Ci, Ci)
    sym = 0.5 * (np.einsum("...AC,...BD->...ABCD", Ci, Ci) + np.einsum("...AD,...BC->...ABCD", Ci, Ci))
    return 2.0 * lam * outer + 2.0 * (mu - 2.0 * lam * lJ[..., None, None, None, None]) * sym


def push_forward(F, CC):
    """chi(CC)_{ijkl} = F_iA F_jB F_kC F_lD CC_ABCD (eq. Jc)."""
    return np.einsum("...iA,...jB,...kC,...lD,...ABCD->...ijkl", F, F, F, F, CC)
