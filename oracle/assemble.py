"""Global assembly, Dirichlet rows and symmetric diagonal scaling (oracle).

Unknown ordering is node-interleaved: dof 4*a + r with r in (vx, vy, vz, p).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import element as E
from . import material as M


class Discretization:
    """Per-mesh constants: reference geometry, tau_M, structure tensors."""

    def __init__(self, mesh, mat):
        self.mesh = mesh
        self.mat = mat
        self.Xe = mesh.X[mesh.tets]
        self.V, self.G = E.ref_geometry(self.Xe)
        self.tau = E.tau_m(self.Xe, mat)
        self.H = None
        if mat.kind == M.HGO_INCOMP:
            self.H = M.structure_tensors(mesh.fibre, mat.kd)
        self.n = mesh.n_nodes
        self.vmask = mesh.dir_mask[:, 0:3].astype(bool)
        self.pmask = mesh.dir_mask[:, 3].astype(bool)
        self.dof_dir = mesh.dir_mask.astype(bool).ravel()

    def gather(self, x):
        return x[self.mesh.tets]

    def nodal_traction(self, scale):
        """-int_Gamma N_A H dGamma for a dead load H = scale * traction, one
        third of each reference face area to each face vertex."""
        f = np.zeros((self.n, 3))
        X = self.mesh.X
        for k, face in enumerate(self.mesh.bfaces):
            a, b, c = X[face]
            area = 0.5 * np.linalg.norm(np.cross(b - a, c - a))
            for node in face:
                f[node] -= scale * self.mesh.traction[k] * area / 3.0
        return f

    def residual(self, st, load_scale):
        """Global (R_m, R_p) as [n][4] at a staged state st (keys dv, dp, u, p, v)."""
        g = self.gather
        Re = E.element_residual(self.V, self.G, self.tau, self.mat, self.H,
                                g(st["dv"]), g(st["dp"]), g(st["u"]), g(st["p"]), g(st["v"]))
        R = np.zeros((self.n, 4))
        np.add.at(R, self.mesh.tets, Re)
        R[:, 0:3] += self.nodal_traction(load_scale)
        return R

    def tangent(self, st, ga):
        """Global reduced tangent [[A, B], [C, D]] (4n x 4n CSR, interleaved)."""
        g = self.gather
        Ke = E.element_tangent(self.V, self.G, self.tau, self.mat, self.H, ga,
                               g(st["dv"]), g(st["dp"]), g(st["u"]), g(st["p"]), g(st["v"]))
        t = self.mesh.tets
        r = 4 * t[:, :, None, None, None] + np.arange(4)[None, None, :, None, None]
        c = 4 * t[:, None, None, :, None] + np.arange(4)[None, None, None, None, :]
        r = np.broadcast_to(r, Ke.shape).ravel()
        c = np.broadcast_to(c, Ke.shape).ravel()
        K = sp.coo_matrix((Ke.ravel(), (r, c)), shape=(4 * self.n, 4 * self.n)).tocsr()
        K.sum_duplicates()
        return K

    def u_jvp(self, st, dirn):
        """Global d(R_m, R_p)/du_{alpha_f} . dirn  ([n][4]); dirn is nodal [n][3]."""
        g = self.gather
        Je = E.element_u_jvp(self.V, self.G, self.tau, self.mat, self.H, g(dirn),
                             g(st["dv"]), g(st["dp"]), g(st["u"]), g(st["p"]), g(st["v"]))
        out = np.zeros((self.n, 4))
        np.add.at(out, self.mesh.tets, Je)
        return out


def apply_dirichlet(K, rhs, dof_dir):
    """Zero the rows and columns of Dirichlet dofs, unit diagonal, zero rhs."""
    keep = sp.diags((~dof_dir).astype(float))
    K = (keep @ K @ keep).tocsr()
    K = K + sp.diags(dof_dir.astype(float))
    rhs = np.where(dof_dir, 0.0, rhs)
    return K.tocsr(), rhs


def scaling(K, eps_diag=1.0e-15):
    """W_ii = |K_ii|^(-1/2) if |K_ii| >= eps_diag else 1 (section 4.1)."""
    d = np.abs(K.diagonal())
    return np.where(d >= eps_diag, 1.0 / np.sqrt(np.where(d > 0, d, 1.0)), 1.0)


def split_blocks(K):
    """[[A, B], [C, D]] sub-blocks of an interleaved 4n x 4n matrix."""
    n4 = K.shape[0]
    idx = np.arange(n4)
    iv = idx[idx % 4 != 3]
    ip = idx[idx % 4 == 3]
    K = K.tocsr()
    return (K[iv][:, iv].tocsr(), K[iv][:, ip].tocsr(),
            K[ip][:, iv].tocsr(), K[ip][:, ip].tocsr(), iv, ip)
