"""Pins for the oracle's element residual and complex-step tangent.

* patch test: an affine deformation with uniform pressure and zero rates,
  loaded on every boundary face by the exact traction (P~ - J p F^-T) N with
  P~ from differentiating the paper's energy, gives R = 0 at every node;
* internal forces of every element sum to zero and carry no moment
  (balance of linear and angular momentum), and the residual is objective;
* the tangent equals central differences of the residual taken through the
  generalized-alpha staging and the stage-2 update (the definition of
  A, B, C, D in the block reduction);
* at rest the blocks reduce to textbook operators: consistent mass plus
  linear deviatoric elasticity (A), the discrete gradient (B), divergence plus
  the tau_M term (C), beta-mass plus the tau_M Laplacian (D).
"""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import assemble as AS
from oracle import element as E
from oracle import material as M
from oracle import newton as NW

H_CS = 1e-30


def energy_piola(F, mu):
    """P = dW/dF for W = mu/2 (tr C~ - 3), by complex step (independent of the oracle)."""
    def W(Fc):
        J = np.linalg.det(Fc)
        return mu / 2 * (J ** (-2 / 3) * np.trace(Fc.T @ Fc) - 3)
    P = np.zeros((3, 3))
    for i in range(3):
        for I in range(3):
            dF = np.zeros((3, 3), dtype=complex)
            dF[i, I] = 1j * H_CS
            P[i, I] = np.imag(W(F + dF)) / H_CS
    return P


def all_boundary_faces(mesh):
    X, T = mesh.X, mesh.tets
    lo = np.isclose(X, 0.0) | np.isclose(X, 1.0)
    faces, normals = [], []
    for d in range(4):
        keep = [a for a in range(4) if a != d]
        f = T[:, keep]
        for ax in range(3):
            on = lo[f, ax].all(axis=1) & np.isclose(X[f[:, 0], ax], X[f[:, 1], ax]) & \
                np.isclose(X[f[:, 0], ax], X[f[:, 2], ax])
            for e in np.nonzero(on)[0]:
                n = np.zeros(3)
                n[ax] = 1.0 if X[f[e, 0], ax] > 0.5 else -1.0
                faces.append(f[e])
                normals.append(n)
    return np.array(faces, dtype=np.int32), np.array(normals)


@pytest.mark.parametrize("N", [2, 4])
def test_patch_test_affine_state(N):
    rng = np.random.default_rng(7)
    mesh, mat, ti = synth.cube_case(N)
    F0 = np.eye(3) + 0.15 * rng.uniform(-1, 1, (3, 3))
    p0 = 2.3e4
    J0 = np.linalg.det(F0)
    P0 = energy_piola(F0, mat.mu)
    faces, normals = all_boundary_faces(mesh)
    trac = (P0 - J0 * p0 * np.linalg.inv(F0).T) @ normals.T
    mesh2 = dataclasses.replace(mesh, bfaces=faces, traction=trac.T.copy())
    disc = AS.Discretization(mesh2, mat)
    n = mesh.n_nodes
    st = {"u": mesh.X @ (F0 - np.eye(3)).T, "p": np.full(n, p0), "v": np.zeros((n, 3)),
          "du": np.zeros((n, 3)), "dp": np.zeros(n), "dv": np.zeros((n, 3))}
    R = disc.residual(st, 1.0)
    scale = np.abs(P0).max() / N ** 2
    assert np.abs(R[:, 0:3]).max() < 1e-9 * scale
    assert np.abs(R[:, 3]).max() < 1e-12


def _random_element_state(mesh, seed):
    st = synth.random_state(mesh.n_nodes, seed)
    return {k: st[k][mesh.tets] for k in st}


def test_internal_forces_balance_and_carry_no_moment():
    mesh, mat, ti = synth.cube_case(3)
    disc = AS.Discretization(mesh, mat)
    st = _random_element_state(mesh, 1)
    zero_dv = np.zeros_like(st["dv"])
    Re = E.element_residual(disc.V, disc.G, disc.tau, mat, None, zero_dv, np.zeros_like(st["dp"]),
                            st["u"], st["p"], np.zeros_like(st["v"]))
    f = Re[:, :, 0:3]
    scale = np.abs(f).max()
    assert np.abs(f.sum(axis=1)).max() < 1e-12 * scale
    x = disc.Xe + st["u"]
    mom = np.cross(x, f).sum(axis=1)
    assert np.abs(mom).max() < 1e-12 * scale
    # the tau_M term of R_p sums to zero over an element's nodes
    assert np.abs(Re[:, :, 3].sum(axis=1)).max() < 1e-12 * np.abs(Re[:, :, 3]).max()


def test_residual_is_objective():
    mesh, mat, ti = synth.cube_case(2)
    disc = AS.Discretization(mesh, mat)
    st = _random_element_state(mesh, 2)
    a = 0.7
    Q = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1.0]])
    Q = Q @ np.array([[1, 0, 0], [0, np.cos(0.3), -np.sin(0.3)], [0, np.sin(0.3), np.cos(0.3)]])
    x = disc.Xe + st["u"]
    u_rot = x @ Q.T - disc.Xe
    R1 = E.element_residual(disc.V, disc.G, disc.tau, mat, None, st["dv"], st["dp"], st["u"], st["p"], st["v"])
    R2 = E.element_residual(disc.V, disc.G, disc.tau, mat, None, st["dv"] @ Q.T, st["dp"], u_rot,
                            st["p"], st["v"] @ Q.T)
    np.testing.assert_allclose(R2[:, :, 0:3], R1[:, :, 0:3] @ Q.T, atol=1e-10 * np.abs(R1[:, :, 0:3]).max())
    np.testing.assert_allclose(R2[:, :, 3], R1[:, :, 3], atol=1e-10 * np.abs(R1[:, :, 3]).max())


@pytest.mark.parametrize("kind", [M.NH_COMP, M.NH_INCOMP])
def test_tangent_matches_fd_through_staging(kind):
    mesh, mat, ti = synth.cube_case(3)
    if kind == M.NH_INCOMP:
        mat = synth.material_from_nu(1e5, 0.5)
    disc = AS.Discretization(mesh, mat)
    am, af, gm = E.genalpha(ti.rho_inf)
    sn = synth.random_state(mesh.n_nodes, 4)
    it = synth.random_state(mesh.n_nodes, 5)
    st = NW.stage(sn, it, am, af)
    K = disc.tangent(st, (am, af, gm, ti.dt))
    rng = np.random.default_rng(9)
    d = rng.standard_normal(4 * mesh.n_nodes)
    d[3::4] *= 1e4   # p-dot directions carry larger magnitudes than v-dot ones
    d[disc.dof_dir] = 0.0   # the update leaves Dirichlet components fixed
    Kd = K @ d

    def R_at(eps):
        zero_rk = np.zeros((mesh.n_nodes, 3))
        it2, _ = NW.newton_update(disc, ti, it, eps * d, zero_rk)
        return disc.residual(NW.stage(sn, it2, am, af), 0.0).ravel()

    eps = 1e-6
    fd = (R_at(eps) - R_at(-eps)) / (2 * eps)
    assert np.linalg.norm(fd - Kd) <= 1e-6 * np.linalg.norm(Kd)


def test_rest_state_blocks_reduce_to_textbook_operators():
    mesh, mat, ti = synth.cube_case(2)
    disc = AS.Discretization(mesh, mat)
    am, af, gm = E.genalpha(ti.rho_inf)
    c2 = af * gm * ti.dt
    c3 = c2 * c2 / am
    m = mesh.n_tets
    z3, z1 = np.zeros((m, 4, 3)), np.zeros((m, 4))
    Ke = E.element_tangent(disc.V, disc.G, disc.tau, mat, None, (am, af, gm, ti.dt), z3, z1, z3, z1, z3)
    mu, rho0, kappa = mat.mu, mat.rho0, mat.kappa
    Dv = mu * np.array([[4 / 3, -2 / 3, -2 / 3, 0, 0, 0], [-2 / 3, 4 / 3, -2 / 3, 0, 0, 0],
                        [-2 / 3, -2 / 3, 4 / 3, 0, 0, 0], [0, 0, 0, 1, 0, 0],
                        [0, 0, 0, 0, 1, 0], [0, 0, 0, 0, 0, 1]])
    for e in range(0, m, 7):
        V, G, tau = disc.V[e], disc.G[e], disc.tau[e]
        Bm = []
        for A in range(4):
            gx, gy, gz = G[A]
            Bm.append(np.array([[gx, 0, 0], [0, gy, 0], [0, 0, gz],
                                [gy, gx, 0], [0, gz, gy], [gz, 0, gx]]))
        for A in range(4):
            for B in range(4):
                mass = V / 20 * (1 + (A == B))
                A_tb = am * rho0 * mass * np.eye(3) + c3 * V * Bm[A].T @ Dv @ Bm[B]
                B_tb = -c2 * V / 4 * G[A]
                C_tb = am * tau * rho0 * V / 4 * G[A] + c2 * V / 4 * G[B]
                D_tb = am / kappa * mass + c2 * tau * V * G[A] @ G[B]
                K = Ke[e, A, :, B, :]
                np.testing.assert_allclose(K[0:3, 0:3], A_tb, rtol=1e-12, atol=1e-12 * np.abs(A_tb).max())
                np.testing.assert_allclose(K[0:3, 3], B_tb, rtol=1e-12, atol=1e-13 * np.abs(B_tb).max())
                np.testing.assert_allclose(K[3, 0:3], C_tb, rtol=1e-12, atol=1e-13 * np.abs(C_tb).max())
                assert K[3, 3] == pytest.approx(D_tb, rel=1e-12, abs=0.0)


def test_tau_m_values():
    # cube 32^3 at nu = 0.45 and 64^3 at nu = 0.499, reference longest edge sqrt(3) h
    for N, nu, expect in ((32, 0.45, 1.63e-9), (64, 0.499, 1.21e-10)):
        mat = synth.material_from_nu(1e5, nu)
        Xe = np.array([[[0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 1]]], dtype=float) / N
        assert E.tau_m(Xe, mat)[0] == pytest.approx(expect, rel=5e-3, abs=0.0)
