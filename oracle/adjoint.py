"""Adjoint gradient of a displacement objective through the time history (oracle).

One time step solves G(y-dot_{n+1}; y_n, y-dot_n, theta) = 0 with
G = (R-bar_k, R_p, R_m) at the generalized-alpha stages (section 3.2 / 3.3) and
y_{n+1} = y_n + dt y-dot_n + gamma dt (y-dot_{n+1} - y-dot_n).  For
J = J(u_N), implicit differentiation at each converged step gives, backwards
from n = N-1 to 0,

    K^T lam = y-dot-bar_{n+1} + gamma dt y-bar_{n+1},   K = dG/dy-dot_{n+1}
    y-bar_n     = y-bar_{n+1}           - lam^T dG/dy_n
    y-dot-bar_n = (1 - gamma) dt y-bar_{n+1} - lam^T dG/dy-dot_n
    dJ/dtheta  -= lam^T dG/dtheta

This module writes that out with no block factorisation: K is the unreduced
3-field tangent (``full3``), solved transposed by sparse LU, and every partial
derivative of G (with respect to y_n, y-dot_n through the stage relations, and
with respect to theta = (mu, kappa, k1, k2, fibre angle)) is taken by complex
step of the residual itself.  Nodal cotangent layout [n][7] = (u 3, p, v 3)
and (u-dot 3, p-dot, v-dot 3).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from synth import fibre_field

from . import assemble as AS
from . import element as E
from . import full3 as F3
from . import material as M
from . import newton as NW

PARAMS = ("mu", "kappa", "k1", "k2", "phi")
H_CS = 1e-30


def with_params(mesh, mat, theta):
    """Mesh and material for theta = (mu, kappa, k1, k2, fibre angle)."""
    mat2 = dataclasses.replace(mat, mu=theta[0], kappa=theta[1], k1=theta[2], k2=theta[3])
    mesh2 = mesh
    if mesh.fibre is not None:
        fib, _ = fibre_field(mesh, theta[4])
        mesh2 = dataclasses.replace(mesh, fibre=fib)
    return mesh2, mat2


def theta_of(mesh, mat):
    phi = mesh.meta.get("fibre_rad", 0.0)
    return np.array([mat.mu, mat.kappa if np.isfinite(mat.kappa) else 0.0, mat.k1, mat.k2, phi])


def forward(mesh, mat, ti, n_steps, tol_R=1e-13):
    """States s_0 .. s_N of the predictor multi-corrector integration."""
    disc = AS.Discretization(mesh, mat)
    states = [NW.rest_state(mesh)]
    for s in range(n_steps):
        st, info = NW.time_step(disc, ti, states[-1], s * ti.dt, tol_R=tol_R, tol_A=1e-300)
        if not info["converged"]:
            raise RuntimeError("oracle forward step did not converge")
        states.append(st)
    return states


def _split7(x):
    return x[..., 0:3], x[..., 3], x[..., 4:7]


def _elem_G(mesh, mat, ti, yn, ydn, yd1):
    """Element residuals (R_m, R_p) [m][4][4] as a function of the gathered
    y_n = (u, p, v), y-dot_n and y-dot_{n+1} (each [m][4][7])."""
    am, af, gm = E.genalpha(ti.rho_inf)
    y1 = yn + ti.dt * ydn + gm * ti.dt * (yd1 - ydn)
    ya = yn + af * (y1 - yn)
    yda = ydn + am * (yd1 - ydn)
    Xe = mesh.X[mesh.tets]
    V, G = E.ref_geometry(Xe)
    tau = E.tau_m(Xe, mat)
    H = M.structure_tensors(mesh.fibre, mat.kd) if mat.kind == M.HGO_INCOMP else None
    u, p, v = _split7(ya)
    _, dp, dv = _split7(yda)
    return E.element_residual(V, G, tau, mat, H, dv, dp, u, p, v)


def _nodal_Rk(ti, yn, ydn, yd1):
    """R-bar_k = u-dot_{n+alpha_m} - v_{n+alpha_f} [n][3]."""
    am, af, gm = E.genalpha(ti.rho_inf)
    y1 = yn + ti.dt * ydn + gm * ti.dt * (yd1 - ydn)
    ya = yn + af * (y1 - yn)
    yda = ydn + am * (yd1 - ydn)
    return yda[:, 0:3] - ya[:, 4:7]


def _pack(st, rates):
    if rates:
        return np.concatenate([st["du"], st["dp"][:, None], st["dv"]], axis=1)
    return np.concatenate([st["u"], st["p"][:, None], st["v"]], axis=1)


def step_cotangents(mesh, mat, ti, sn, s1, lam):
    """lam^T dG/dy_n and lam^T dG/dy-dot_n ([n][7] each) by complex step.

    lam [n][7] has the equation layout of ``full3``: (R-bar_k 3, R_p, R_m 3)."""
    n = mesh.n_nodes
    t = mesh.tets
    yn, ydn, yd1 = _pack(sn, False), _pack(sn, True), _pack(s1, True)
    lam_k, lam_p, lam_m = lam[:, 0:3], lam[:, 3], lam[:, 4:7]
    le_m, le_p = lam_m[t], lam_p[t]
    out = []
    for which in (0, 1):               # 0: y_n, 1: y-dot_n
        cot = np.zeros((n, 7))
        for a in range(4):
            for f in range(7):
                args = [yn[t].astype(complex), ydn[t].astype(complex), yd1[t].astype(complex)]
                args[which][:, a, f] += 1j * H_CS
                R = _elem_G(mesh, mat, ti, *args).imag / H_CS
                contrib = np.einsum("mai,mai->m", le_m, R[:, :, 0:3]) + np.einsum("ma,ma->m", le_p, R[:, :, 3])
                np.add.at(cot[:, f], t[:, a], contrib)
        for f in range(7):             # kinematic rows (nodal)
            args = [yn.astype(complex), ydn.astype(complex), yd1.astype(complex)]
            args[which][:, f] += 1j * H_CS
            dRk = _nodal_Rk(ti, *args).imag / H_CS
            cot[:, f] += np.einsum("ni,ni->n", lam_k, dRk)
        out.append(cot)
    return out[0], out[1]


def theta_cotangent(mesh, mat, ti, theta, sn, s1, lam, k):
    """lam^T dG/dtheta_k by complex step in theta_k (R-bar_k has no theta)."""
    th = np.asarray(theta, dtype=complex).copy()
    th[k] += 1j * H_CS
    mesh_c, mat_c = with_params(mesh, mat, th)
    t = mesh.tets
    yn, ydn, yd1 = _pack(sn, False)[t], _pack(sn, True)[t], _pack(s1, True)[t]
    R = _elem_G(mesh_c, mat_c, ti, yn.astype(complex), ydn.astype(complex), yd1.astype(complex)).imag / H_CS
    lam_p, lam_m = lam[:, 3][t], lam[:, 4:7][t]
    return float(np.sum(lam_m * R[:, :, 0:3]) + np.sum(lam_p * R[:, :, 3]))


def backward_step(mesh, mat, ti, theta, sn, s1, ybar, ydbar, params=(0, 1)):
    """One step of the recursion: returns (y-bar_n, y-dot-bar_n, -lam^T dG/dtheta, lam)."""
    mesh_t, mat_t = with_params(mesh, mat, theta)
    disc = AS.Discretization(mesh_t, mat_t)
    am, af, gm = E.genalpha(ti.rho_inf)
    n = mesh.n_nodes
    mask = np.zeros((n, 7), dtype=bool)
    mask[:, 0:3] = disc.vmask
    mask[:, 3] = disc.pmask
    mask[:, 4:7] = disc.vmask
    d = mask.ravel()
    keep = sp.diags((~d).astype(float))
    st = NW.stage(sn, s1, am, af)
    Kf, _ = F3.full_system(disc, ti, st, 0.0)
    Kd = (keep @ Kf @ keep + sp.diags(d.astype(float))).tocsc()
    g = ydbar + gm * ti.dt * ybar
    g[mask] = 0.0
    lam = spla.splu(Kd.T.tocsc()).solve(g.ravel()).reshape(n, 7)
    cot_y, cot_yd = step_cotangents(mesh_t, mat_t, ti, sn, s1, lam)
    dth = np.zeros(5)
    for k in params:
        dth[k] = -theta_cotangent(mesh, mat, ti, theta, sn, s1, lam, k)
    return ybar - cot_y, (1.0 - gm) * ti.dt * ybar - cot_yd, dth, lam


def adjoint_gradient(mesh, mat, ti, theta, states, dJdu, params=(0, 1)):
    """dJ/dtheta for J = J(u_N) with dJ/du_N = dJdu [n][3]."""
    n = mesh.n_nodes
    ybar = np.zeros((n, 7))
    ybar[:, 0:3] = dJdu
    ydbar = np.zeros((n, 7))
    grad = np.zeros(5)
    for s in range(len(states) - 2, -1, -1):
        ybar, ydbar, dth, _ = backward_step(mesh, mat, ti, theta, states[s], states[s + 1], ybar, ydbar, params)
        grad += dth
    return grad


def objective(u, sel, u_target):
    """J = 1/2 || u[sel] - u_target ||^2 and dJ/du."""
    diff = u[sel] - u_target
    dJ = np.zeros_like(u)
    dJ[sel] = diff
    return 0.5 * float(np.sum(diff * diff)), dJ
