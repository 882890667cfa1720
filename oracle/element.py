"""Element-level residuals and tangents for P1 tetrahedra (oracle).

Residuals follow the consistent-linearization appendix (R_p, R_m written on
the reference configuration), with the P1 simplifications that F is constant
per element (so the divergence of P~ vanishes) and body force b = 0.
Integrals use the symmetric 4-point degree-2 tetrahedral rule (weights V/4)
for every term.

Tangents are not taken from the appendix' closed forms: they are the exact
derivatives of these residuals along the generalized-alpha kinematics, taken
by complex-step differentiation.  The column for a rate unknown y-dot_{n+1}
moves the alpha_m-stage rate by alpha_m, the alpha_f-stage value by
alpha_f*gamma*dt and (for velocity rates, through the kinematic stage-2
relation Delta u-dot = (alpha_f gamma dt/alpha_m) Delta v-dot) the
displacement by (alpha_f gamma dt)^2/alpha_m -- the definitions of A, B, C,
D in the block reduction of the Newton system (section 3.3).
"""
from __future__ import annotations

import numpy as np

from . import material as M

QA = 0.5854101966249685   # (5 + 3 sqrt 5)/20
QB = 0.1381966011250105   # (5 - sqrt 5)/20
NQ = np.full((4, 4), QB)
np.fill_diagonal(NQ, QA)  # NQ[q, A] = N_A at quadrature point q

CS_H = 1.0e-30            # complex-step size


def genalpha(rho_inf: float):
    """alpha_m, alpha_f, gamma for first-order systems (section 3.2)."""
    am = 0.5 * (3.0 - rho_inf) / (1.0 + rho_inf)
    af = 1.0 / (1.0 + rho_inf)
    return am, af, af


def ref_geometry(Xe):
    """Reference volume V and reference shape-function gradients G[m][A][I]."""
    Mx = np.swapaxes(Xe[:, 1:, :] - Xe[:, 0:1, :], 1, 2)   # columns are edges
    V = np.linalg.det(Mx) / 6.0
    Minv = np.linalg.inv(Mx)                                # row a = grad xi_a
    G = np.empty((Xe.shape[0], 4, 3))
    G[:, 1:, :] = Minv
    G[:, 0, :] = -Minv.sum(axis=1)
    return V, G


def tau_m(Xe, mat):
    """tau_M = c_m h_e / (c rho) (section 3.1), frozen per element: h_e is the
    longest reference edge (the diameter of a tetrahedron) and rho -> rho0."""
    h = np.zeros(Xe.shape[0])
    for a in range(4):
        for b in range(a + 1, 4):
            h = np.maximum(h, np.linalg.norm(Xe[:, a] - Xe[:, b], axis=1))
    return mat.c_m * h / (M.wave_speed(mat) * mat.rho0)


def element_residual(V, G, tau, mat, H, dv, dp, u, p, v):
    """Element residual [m][A][4] = (R_m^x, R_m^y, R_m^z, R_p) at node A.

    dv, dp are the alpha_m-stage rates v-dot, p-dot; u, p, v the alpha_f-stage
    values; all gathered per element ([m][4][3] or [m][4]).
    """
    m = V.shape[0]
    eye = np.eye(3)
    F = eye[None] + np.einsum("mai,maI->miI", u, G)
    J = np.linalg.det(F)
    Finv = np.linalg.inv(F)
    g = np.einsum("maI,mIi->mai", G, Finv)          # spatial gradients N_A,i
    divv = np.einsum("mai,mai->m", v, g)
    gradp = np.einsum("ma,mai->mi", p, g)
    pq = np.einsum("qa,ma->mq", NQ, p)
    dpq = np.einsum("qa,ma->mq", NQ, dp)
    dvq = np.einsum("qa,mai->mqi", NQ, dv)
    rho, beta, _, _ = M.rho_beta(pq, mat)
    P = M.piola_iso(F, mat, H)
    w = V / 4.0

    R = np.zeros((m, 4, 4), dtype=np.result_type(u, dv, p, dp, v))
    # momentum: int N_A J rho v-dot_i + N_A,I P~_iI - N_A,i J p
    for q in range(4):
        R[:, :, 0:3] += (w * J)[:, None, None] * NQ[q][None, :, None] * \
            (rho[:, q, None] * dvq[:, q, :])[:, None, :]
        R[:, :, 0:3] += w[:, None, None] * np.einsum("miI,maI->mai", P, G)
        R[:, :, 0:3] -= (w * J * pq[:, q])[:, None, None] * g
    # mass: int J N_A (beta p-dot + v_i,i) + tau N_A,i (rho J v-dot_i + J p_,i)
    for q in range(4):
        R[:, :, 3] += (w * J)[:, None] * NQ[q][None, :] * (beta[:, q] * dpq[:, q] + divv)[:, None]
        stab = rho[:, q, None] * dvq[:, q, :] + gradp
        R[:, :, 3] += (w * tau * J)[:, None] * np.einsum("mai,mi->ma", g, stab)
    return R


def element_tangent(V, G, tau, mat, H, ga, dv, dp, u, p, v):
    """Element blocks of the reduced tangent [[A, B], [C, D]] by complex step.

    Returns K[m][A][r][B][c] with r, c in (vx, vy, vz, p): K[.., 0:3, .., 0:3]
    is A, [.., 0:3, .., 3] is B, [.., 3, .., 0:3] is C, [.., 3, .., 3] is D.
    ``ga`` = (alpha_m, alpha_f, gamma, dt).
    """
    am, af, gm, dt = ga
    c2 = af * gm * dt
    c3 = c2 * c2 / am
    m = V.shape[0]
    K = np.zeros((m, 4, 4, 4, 4))
    ih = 1j * CS_H
    for B in range(4):
        for c in range(4):
            dvc, dpc, uc, pc, vc = (x.astype(complex) for x in (dv, dp, u, p, v))
            if c < 3:
                dvc[:, B, c] += am * ih
                vc[:, B, c] += c2 * ih
                uc[:, B, c] += c3 * ih
            else:
                dpc[:, B] += am * ih
                pc[:, B] += c2 * ih
            R = element_residual(V, G, tau, mat, H, dvc, dpc, uc, pc, vc)
            K[:, :, :, B, c] = R.imag / CS_H
    return K


def element_u_jvp(V, G, tau, mat, H, dirn, dv, dp, u, p, v):
    """Directional derivative of the element residual with respect to the
    alpha_f-stage displacement along ``dirn`` ([m][4][3]), by complex step."""
    uc = u.astype(complex) + 1j * CS_H * dirn
    R = element_residual(V, G, tau, mat, H, dv.astype(complex), dp.astype(complex),
                         uc, p.astype(complex), v.astype(complex))
    return R.imag / CS_H
