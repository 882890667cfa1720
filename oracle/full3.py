"""The unreduced 3-field Newton system (section 3.3), oracle.

Unknowns per node: (u-dot 3, p-dot 1, v-dot 3); equations per node:
(R-bar_k 3, R_p 1, R_m 3), with R-bar_k = u-dot_{n+alpha_m} - v_{n+alpha_f}.
Its tangent K is taken by complex step along the generalized-alpha stage
relations, without the block factorization, so that the two-stage reduced
solve can be checked against it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import element as E


def full_system(disc, ti, st, load):
    am, af, gm = E.genalpha(ti.rho_inf)
    c2 = af * gm * ti.dt
    n = disc.n
    g = disc.gather
    dv, dp, u, p, v = (g(st[k]) for k in ("dv", "dp", "u", "p", "v"))
    m = dv.shape[0]
    Rk = st["du"] - st["v"]
    R = disc.residual(st, load)
    Rfull = np.zeros((n, 7))
    Rfull[:, 0:3] = Rk
    Rfull[:, 3] = R[:, 3]
    Rfull[:, 4:7] = R[:, 0:3]

    ih = 1j * E.CS_H
    Ke = np.zeros((m, 4, 7, 4, 7))     # rows (R_m xyz, R_p) mapped below
    for B in range(4):
        for c in range(7):
            dvc, dpc, uc, pc, vc = (x.astype(complex) for x in (dv, dp, u, p, v))
            if c < 3:                  # u-dot: moves u_{alpha_f} by alpha_f gamma dt
                uc[:, B, c] += c2 * ih
            elif c == 3:               # p-dot
                dpc[:, B] += am * ih
                pc[:, B] += c2 * ih
            else:                      # v-dot
                dvc[:, B, c - 4] += am * ih
                vc[:, B, c - 4] += c2 * ih
            Re = E.element_residual(disc.V, disc.G, disc.tau, disc.mat, disc.H,
                                    dvc, dpc, uc, pc, vc).imag / E.CS_H
            Ke[:, :, 3, B, c] = Re[:, :, 3]
            Ke[:, :, 4:7, B, c] = Re[:, :, 0:3]
    t = disc.mesh.tets
    r = 7 * t[:, :, None, None, None] + np.arange(7)[None, None, :, None, None]
    cc = 7 * t[:, None, None, :, None] + np.arange(7)[None, None, None, None, :]
    rows = [np.broadcast_to(r, Ke.shape).ravel()]
    cols = [np.broadcast_to(cc, Ke.shape).ravel()]
    vals = [Ke.ravel()]
    # kinematic rows: d R-bar_k / d u-dot = alpha_m I, d R-bar_k / d v-dot = -af g dt I
    a = np.arange(n)
    for i in range(3):
        rows += [7 * a + i, 7 * a + i]
        cols += [7 * a + i, 7 * a + 4 + i]
        vals += [np.full(n, am), np.full(n, -c2)]
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(7 * n, 7 * n)).tocsr()
    return K, Rfull


def solve_full(disc, K, Rfull):
    """Solve K Delta = -R with Dirichlet rows (u-dot, v-dot on fixed velocity
    components, p-dot on fixed pressures); returns du, dp, dv increments."""
    n = disc.n
    mask = np.zeros((n, 7), dtype=bool)
    mask[:, 0:3] = disc.vmask
    mask[:, 3] = disc.pmask
    mask[:, 4:7] = disc.vmask
    d = mask.ravel()
    keep = sp.diags((~d).astype(float))
    Kd = (keep @ K @ keep + sp.diags(d.astype(float))).tocsc()
    rhs = np.where(d, 0.0, -Rfull.ravel())
    x = spla.splu(Kd).solve(rhs).reshape(n, 7)
    return {"du": x[:, 0:3], "dp": x[:, 3], "dv": x[:, 4:7]}
