"""Constitutive relations (section 2 and the numerical-results section).

All functions accept complex arrays so that complex-step differentiation can
run through them; nothing here takes an absolute value or a conjugate.
"""
from __future__ import annotations

import numpy as np

NH_COMP, NH_INCOMP, HGO_INCOMP = 0, 1, 2


def rho_beta(p, mat):
    """rho(p) = (dG_vol/dp)^-1 and beta(p) = rho^-1 d rho/dp (section 2),
    plus d rho/dp and d beta/dp.

    For the volumetric Gibbs energy of the block-compression example,
    G_vol = (p s - p^2)/(2 kappa rho0) - kappa/(2 rho0) ln((s - p)/kappa) with
    s = sqrt(p^2 + kappa^2), dG_vol/dp = (s - p)/(kappa rho0), hence
    rho = rho0 (s + p)/kappa, beta = 1/s, rho_p = rho beta, beta_p = -p/s^3.
    The fully incompressible energy G_vol = p/rho0 gives rho = rho0, beta = 0.
    """
    p = np.asarray(p)
    if mat.kind == NH_COMP:
        s = np.sqrt(p * p + mat.kappa * mat.kappa)
        rho = mat.rho0 * (s + p) / mat.kappa
        beta = 1.0 / s
        return rho, beta, rho * beta, -p / (s * s * s)
    z = np.zeros_like(p)
    return z + mat.rho0, z, z, z


def wave_speed(mat) -> float:
    """c in tau_M (section 3.1): bulk wave speed sqrt((lambda + 2 mu)/rho0) for
    compressible materials (lambda + 2 mu = kappa + 4 mu / 3), shear wave speed
    sqrt(mu/rho0) for incompressible ones."""
    if mat.kind == NH_COMP:
        return np.sqrt((mat.kappa + 4.0 * mat.mu / 3.0) / mat.rho0)
    return np.sqrt(mat.mu / mat.rho0)


def structure_tensors(fibre, kd):
    """H_i = k_d I + (1 - 3 k_d) a_i (x) a_i for the two fibre families
    (anisotropic tensile test).  fibre: [m][2][3] -> [m][2][3][3]."""
    a = np.asarray(fibre)
    eye = np.eye(3)
    return kd * eye[None, None] + (1.0 - 3.0 * kd) * np.einsum("mfi,mfj->mfij", a, a)


def piola_iso(F, mat, H=None):
    """Iso first Piola stress P~ = d(rho0 G_iso)/dF = J sigma_dev F^-T.

    neo-Hookean: mu J^(-2/3) (F - tr(C)/3 F^-T).
    fibre i:     2 k1 E_i exp(k2 E_i^2) J^(-2/3) (F H_i - (H_i : C)/3 F^-T).
    """
    J = np.linalg.det(F)
    Finv = np.linalg.inv(F)
    FinvT = np.swapaxes(Finv, -1, -2)
    C = np.einsum("...kI,...kJ->...IJ", F, F)
    trC = np.einsum("...II->...", C)
    Jm23 = J ** (-2.0 / 3.0)
    P = mat.mu * Jm23[..., None, None] * (F - trC[..., None, None] / 3.0 * FinvT)
    if mat.kind == HGO_INCOMP and H is not None:
        for f in range(2):
            Hf = H[..., f, :, :]
            HC = np.einsum("...IJ,...IJ->...", Hf, C)
            E = Jm23 * HC - 1.0
            coef = 2.0 * mat.k1 * E * np.exp(mat.k2 * E * E) * Jm23
            P = P + coef[..., None, None] * (np.einsum("...iK,...KI->...iI", F, Hf)
                                             - HC[..., None, None] / 3.0 * FinvT)
    return P
