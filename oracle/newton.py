"""Generalized-alpha predictor multi-corrector time step (section 3.3), oracle.

State dictionaries hold nodal arrays: u, v [n][3], p [n] and their rates
du, dv [n][3], dp [n].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import assemble as AS
from .element import genalpha

KEYS_VAL = ("u", "p", "v")
KEYS_RATE = ("du", "dp", "dv")


def rest_state(mesh):
    """Start from rest; prescribed-velocity Dirichlet components move from t = 0."""
    n = mesh.n_nodes
    st = {"u": np.zeros((n, 3)), "p": np.zeros(n), "v": np.zeros((n, 3)),
          "du": np.zeros((n, 3)), "dp": np.zeros(n), "dv": np.zeros((n, 3))}
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    st["v"][vm] = mesh.dir_vel[vm]
    st["du"][vm] = mesh.dir_vel[vm]
    return st


def predictor(mesh, state_n, gm, t_np1, lift=False):
    """y_(0) = y_n, y-dot_(0) = (gamma - 1)/gamma y-dot_n (section 3.3, predictor
    stage).  Preset form (lift=False): the Dirichlet components take their
    prescribed motion u = g(t), v = g-dot(t), v-dot = 0 at once.  Lifted form
    (lift=True): every node takes the predictor, v-dot = 0 on the Dirichlet
    components, and the prescribed displacement arrives through R-bar_k in the
    first corrector (newton_update)."""
    it = {k: state_n[k].copy() for k in KEYS_VAL}
    for k in KEYS_RATE:
        it[k] = (gm - 1.0) / gm * state_n[k]
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    if lift:
        it["dv"][vm] = 0.0
        return it
    it["u"][vm] = (mesh.dir_vel * t_np1)[vm]
    it["v"][vm] = mesh.dir_vel[vm]
    it["du"][vm] = mesh.dir_vel[vm]
    it["dv"][vm] = 0.0
    return it


def stage(state_n, it, am, af):
    """y-dot_{n+alpha_m} = y-dot_n + alpha_m (y-dot_(l-1) - y-dot_n),
    y_{n+alpha_f} = y_n + alpha_f (y_(l-1) - y_n)."""
    st = {}
    for k in KEYS_RATE:
        st[k] = state_n[k] + am * (it[k] - state_n[k])
    for k in KEYS_VAL:
        st[k] = state_n[k] + af * (it[k] - state_n[k])
    return st


def load_scale(ti, t):
    """Dead load ramps linearly in time to full at n_steps * dt."""
    return min(t / (ti.n_steps * ti.dt), 1.0)


def residual_norm(disc, R, Rk):
    """l2 norm of {R-bar_k, R_p, R_m} over the non-Dirichlet dofs."""
    vm, pm = disc.vmask, disc.pmask
    s = np.sum(Rk[~vm] ** 2) + np.sum(R[:, 0:3][~vm] ** 2) + np.sum(R[:, 3][~pm] ** 2)
    return float(np.sqrt(s))


def linear_system(disc, ti, st, load, rk_corr=True):
    """Assemble the stage-1 system of the block reduction (section 3.3):
    K = [[A, B], [C, D]] and rhs = -[R_m - K_m,u-dot R-bar_k/alpha_m;
    R_p - K_p,u-dot R-bar_k/alpha_m], before Dirichlet rows and scaling."""
    am, af, gm = genalpha(ti.rho_inf)
    c2 = af * gm * ti.dt
    Rk = st["du"] - st["v"]
    R = disc.residual(st, load)
    K = disc.tangent(st, (am, af, gm, ti.dt))
    rhs = -R.ravel()
    if rk_corr:
        rhs = rhs + (c2 / am) * disc.u_jvp(st, Rk).ravel()
    return K, rhs, R, Rk


def solve_scaled(K, rhs, dof_dir, eps_diag=1.0e-15, scaled=True):
    """Dirichlet rows, symmetric diagonal scaling, sparse LU: Delta = W x*,
    (W K W) x* = W rhs (section 4.1)."""
    Kd, rd = AS.apply_dirichlet(K, rhs, dof_dir)
    if not scaled:
        return spla.splu(Kd.tocsc()).solve(rd)
    W = AS.scaling(Kd, eps_diag)
    Ks = (Kd.multiply(W[:, None]).multiply(W[None, :])).tocsc()
    xs = spla.splu(Ks).solve(W * rd)
    return W * xs


def newton_update(disc, ti, it, x, Rk, lift=False):
    """Stage 2 and the update: Delta u-dot = (af g dt/am) Delta v-dot - R-bar_k/am;
    y-dot_(l) = y-dot_(l-1) + Delta y-dot; y_(l) = y_(l-1) + gamma dt Delta y-dot.
    Delta v-dot = 0 on Dirichlet components.  Preset form: Delta u-dot = 0 there
    too.  Lifted form: Delta u-dot = -R-bar_k/am there, which carries u to
    g(t_{n+1}) in the first corrector."""
    am, af, gm = genalpha(ti.rho_inf)
    c2 = af * gm * ti.dt
    n = disc.n
    x = x.reshape(n, 4)
    d = {"dv": x[:, 0:3].copy(), "dp": x[:, 3].copy()}
    d["dv"][disc.vmask] = 0.0
    d["dp"][disc.pmask] = 0.0
    d["du"] = (c2 / am) * d["dv"] - Rk / am
    if not lift:
        d["du"][disc.vmask] = 0.0
    out = {}
    for rk, vk in (("du", "u"), ("dp", "p"), ("dv", "v")):
        out[rk] = it[rk] + d[rk]
        out[vk] = it[vk] + gm * ti.dt * d[rk]
    return out, d


def time_step(disc, ti, state_n, t_n, tol_R=1e-10, tol_A=1e-50, l_max=20,
              rk_corr=True, solver=None, lift=False):
    """One generalized-alpha step by the predictor multi-corrector algorithm.

    ``solver(K, rhs, dof_dir) -> Delta`` defaults to the scaled sparse LU.
    ``lift`` selects the lifted Dirichlet predictor (predictor, newton_update);
    it needs rk_corr, whose right-hand-side term K_{.,u-dot} R-bar_k / alpha_m
    then spreads the boundary motion into the interior.  Its relative Newton
    test divides by the largest residual norm of the iterates so far, since the
    predictor's residual does not yet hold the prescribed motion.
    Returns (state_{n+1}, info) with the residual history and a flag.
    """
    if lift and not rk_corr:
        raise ValueError("the lifted Dirichlet predictor needs rk_corr")
    am, af, gm = genalpha(ti.rho_inf)
    solver = solver or solve_scaled
    t_np1 = t_n + ti.dt
    load = load_scale(ti, t_n + af * ti.dt)
    it = predictor(disc.mesh, state_n, gm, t_np1, lift)
    norms, R0, converged = [], None, False
    for l in range(1, l_max + 1):
        st = stage(state_n, it, am, af)
        Rk = st["du"] - st["v"]
        R = disc.residual(st, load)
        nrm = residual_norm(disc, R, Rk)
        norms.append(nrm)
        if R0 is None:
            R0 = nrm
        if lift:
            # the predictor's residual lacks the prescribed motion, which arrives with the first
            # corrector: the reference is the largest residual of the iterates so far
            R0 = max(R0, nrm)
        if (R0 > 0 and nrm / R0 <= tol_R) or nrm <= tol_A:
            converged = True
            break
        K, rhs, _, _ = linear_system(disc, ti, st, load, rk_corr)
        x = solver(K, rhs, disc.dof_dir)
        it, _ = newton_update(disc, ti, it, x, Rk, lift)
    return it, {"norms": norms, "converged": converged, "n_newton": len(norms) - 1}
