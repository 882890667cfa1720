"""Pins for the oracle's time step (section 3.3) and linear algebra (section 4).

* the two-stage reduced solve equals the unreduced 3-field Newton solve;
* after a Newton update the kinematic residual R-bar_k vanishes;
* Newton converges quadratically with the complex-step tangent;
* a rigid translation is integrated exactly (u = u0 + v0 t, v = v0);
* symmetric diagonal scaling leaves the solution unchanged;
* sparse LU, plain GMRES and FGMRES with the exact block preconditioners agree,
  and the exact LDU preconditioner gives one FGMRES iteration, the upper and
  lower triangular ones at most two (the remark on partial factorizations);
* the matrix-free Schur product (Algorithm 2) equals the dense D - C A^-1 B.
"""
import dataclasses

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import assemble as AS
from oracle import element as E
from oracle import full3 as F3
from oracle import krylov as KR
from oracle import newton as NW


def _nonzero_iterate(mesh, ti, seed):
    """A state after a loaded step (so R-bar_k of the next predictor is nonzero)."""
    sn = synth.random_state(mesh.n_nodes, seed)
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    for k in ("u", "v", "du", "dv"):
        sn[k][vm] = 0.0
    am, af, gm = E.genalpha(ti.rho_inf)
    it = NW.predictor(mesh, sn, gm, ti.dt)
    return sn, it, NW.stage(sn, it, am, af)


@pytest.mark.parametrize("kind", ["comp", "incomp"])
def test_reduced_solve_equals_full_three_field_solve(kind):
    mesh, mat, ti = synth.cube_case(3)
    if kind == "incomp":
        mat = synth.material_from_nu(1e5, 0.5)
    disc = AS.Discretization(mesh, mat)
    sn, it, st = _nonzero_iterate(mesh, ti, 21)
    Rk = st["du"] - st["v"]
    assert np.abs(Rk).max() > 1e-3
    K, rhs, R, _ = NW.linear_system(disc, ti, st, 0.5, rk_corr=True)
    x = NW.solve_scaled(K, rhs, disc.dof_dir)
    _, d = NW.newton_update(disc, ti, it, x, Rk)
    Kf, Rf = F3.full_system(disc, ti, st, 0.5)
    df = F3.solve_full(disc, Kf, Rf)
    for key in ("du", "dp", "dv"):
        np.testing.assert_allclose(d[key], df[key], rtol=1e-9, atol=1e-10 * np.abs(df[key]).max())


def test_kinematic_residual_vanishes_after_update():
    mesh, mat, ti = synth.cube_case(3)
    disc = AS.Discretization(mesh, mat)
    am, af, gm = E.genalpha(ti.rho_inf)
    sn, it, st = _nonzero_iterate(mesh, ti, 22)
    Rk = st["du"] - st["v"]
    K, rhs, _, _ = NW.linear_system(disc, ti, st, 0.5)
    x = NW.solve_scaled(K, rhs, disc.dof_dir)
    it2, _ = NW.newton_update(disc, ti, it, x, Rk)
    st2 = NW.stage(sn, it2, am, af)
    Rk2 = st2["du"] - st2["v"]
    assert np.abs(Rk2).max() <= 1e-14 * np.abs(Rk).max() + 1e-300


@pytest.mark.parametrize("nu", [0.3, 0.45, 0.499, 0.5])
def test_newton_converges_quadratically(nu):
    mesh, mat, ti = synth.cube_case(3, nu=nu, dt=5e-3, n_steps=1)
    mesh = dataclasses.replace(mesh, traction=mesh.traction * 40.0)   # strongly nonlinear load
    disc = AS.Discretization(mesh, mat)
    st, info = NW.time_step(disc, ti, NW.rest_state(mesh), 0.0, tol_R=1e-13)
    r = np.array(info["norms"])
    assert info["converged"] and len(r) <= 8
    # at least one step in the asymptotic range shows e_{l+1} ~ C e_l^2:
    # the log-ratio slope log(r_{l+1}/r_l)/log(r_l/r_{l-1}) approaches 2
    slopes = [np.log(r[k + 1] / r[k]) / np.log(r[k] / r[k - 1]) for k in range(1, len(r) - 1)
              if r[k + 1] > 1e-12 * r[0]]
    assert max(slopes) > 1.8


def test_multistep_keeps_quadratic_convergence_with_rk_correction():
    mesh, mat, ti = synth.cube_case(3, nu=0.45, n_steps=3)
    disc = AS.Discretization(mesh, mat)
    st = NW.rest_state(mesh)
    for n in range(3):
        st, info = NW.time_step(disc, ti, st, n * ti.dt, tol_R=1e-12)
        assert info["converged"] and info["n_newton"] <= 3


def test_rigid_translation_is_exact():
    mesh, mat, ti = synth.cube_case(2, n_steps=4)
    mesh = dataclasses.replace(mesh, bfaces=mesh.bfaces[:0], traction=mesh.traction[:0],
                               dir_mask=np.zeros_like(mesh.dir_mask))
    disc = AS.Discretization(mesh, mat)
    v0 = np.array([0.3, -1.2, 0.7])
    st = NW.rest_state(mesh)
    st["v"][:] = v0
    st["du"][:] = v0
    t = 0.0
    for _ in range(4):
        st, info = NW.time_step(disc, ti, st, t, tol_R=1e-14, tol_A=1e-12)
        t += ti.dt
        assert info["converged"]
    np.testing.assert_allclose(st["u"], np.tile(v0 * t, (mesh.n_nodes, 1)), rtol=1e-12)
    np.testing.assert_allclose(st["v"], np.tile(v0, (mesh.n_nodes, 1)), rtol=1e-12)
    assert np.abs(st["p"]).max() < 1e-6 and np.abs(st["dv"]).max() < 1e-6


def test_symmetric_scaling_does_not_change_the_solution():
    mesh, mat, ti = synth.cube_case(3)
    disc = AS.Discretization(mesh, mat)
    _, _, st = _nonzero_iterate(mesh, ti, 23)
    K, rhs, _, _ = NW.linear_system(disc, ti, st, 0.5)
    x1 = NW.solve_scaled(K, rhs, disc.dof_dir, scaled=True)
    x2 = NW.solve_scaled(K, rhs, disc.dof_dir, scaled=False)
    np.testing.assert_allclose(x1, x2, rtol=1e-9, atol=1e-12 * np.abs(x2).max())


def _scaled_blocks(N=3, seed=24, nu=None):
    mesh, mat, ti = synth.cube_case(N, nu=nu)
    disc = AS.Discretization(mesh, mat)
    _, _, st = _nonzero_iterate(mesh, ti, seed)
    K, rhs, _, _ = NW.linear_system(disc, ti, st, 0.5)
    Kd, rd = AS.apply_dirichlet(K, rhs, disc.dof_dir)
    W = AS.scaling(Kd)
    Ks = Kd.multiply(W[:, None]).multiply(W[None, :]).tocsr()
    return Ks, W * rd


def test_gmres_and_lu_agree():
    Ks, r = _scaled_blocks()
    x_lu = spla.splu(Ks.tocsc()).solve(r)
    x_gm, its, _ = KR.fgmres(lambda z: Ks @ z, r, None, rtol=1e-13, maxit=Ks.shape[0])
    np.testing.assert_allclose(x_gm, x_lu, rtol=1e-7, atol=1e-9 * np.abs(x_lu).max())
    # textbook GMRES on a dense system
    rng = np.random.default_rng(0)
    Md = np.eye(30) * 4 + rng.standard_normal((30, 30))
    b = rng.standard_normal(30)
    x, k, _ = KR.fgmres(lambda z: Md @ z, b, rtol=1e-14, maxit=30)
    np.testing.assert_allclose(x, np.linalg.solve(Md, b), rtol=1e-10)


@pytest.mark.parametrize("variant,max_its", [("ldu", 1), ("upper", 2), ("lower", 2)])
@pytest.mark.parametrize("nu", [0.45, 0.5])
def test_exact_block_preconditioner_iteration_counts(variant, max_its, nu):
    Ks, r = _scaled_blocks(nu=nu)
    A, B, C, D, iv, ip = AS.split_blocks(Ks)
    perm = np.concatenate([iv, ip])
    Kp = Ks[perm][:, perm].tocsr()
    rp = r[perm]
    P = KR.block_preconditioner(A, B, C, D, variant)
    x, its, hist = KR.fgmres(lambda z: Kp @ z, rp, P, rtol=1e-10, maxit=20)
    assert its <= max_its
    x_lu = spla.splu(Kp.tocsc()).solve(rp)
    np.testing.assert_allclose(x, x_lu, rtol=1e-8, atol=1e-10 * np.abs(x_lu).max())


def test_block_diagonal_preconditioner_is_not_bounded_by_four_when_D_nonzero():
    # With D != 0 the block-diagonal form has no small iteration bound; only
    # check that it still converges (the LDU/upper bounds are the invariants).
    Ks, r = _scaled_blocks()
    A, B, C, D, iv, ip = AS.split_blocks(Ks)
    perm = np.concatenate([iv, ip])
    Kp = Ks[perm][:, perm].tocsr()
    P = KR.block_preconditioner(A, B, C, D, "diag")
    x, its, _ = KR.fgmres(lambda z: Kp @ z, r[perm], P, rtol=1e-10, maxit=400)
    assert np.linalg.norm(Kp @ x - r[perm]) <= 1e-9 * np.linalg.norm(r)


def test_matrix_free_schur_equals_dense():
    Ks, _ = _scaled_blocks()
    A, B, C, D, _, _ = AS.split_blocks(Ks)
    S = KR.schur_dense(A, B, C, D)
    xp = np.random.default_rng(3).standard_normal(D.shape[0])
    np.testing.assert_allclose(KR.schur_apply_matrix_free(A, B, C, D, xp), S @ xp,
                               rtol=1e-10, atol=1e-12 * np.abs(S @ xp).max())


@pytest.mark.parametrize("nu", [0.3, 0.499])
def test_velocity_block_is_symmetric_without_acceleration(nu):
    """A = dR_m/d(v-dot) is the mass term plus c3 times the second derivative
    of the stored energy and of the pressure work, both symmetric, plus the
    inertial term N_A rho v-dot_i dJ/du (no body force here).  So A is
    symmetric when v-dot = 0, and its skew part is linear in v-dot (section
    3.3 definition of A; App. A).  A transposed or dropped stiffness term
    breaks the first property, a misplaced inertial term the second."""
    mesh, mat, ti = synth.cube_case(3, nu=nu)
    disc = AS.Discretization(mesh, mat)
    am, af, gm = E.genalpha(ti.rho_inf)
    skew = []
    for scale in (0.0, 1.0, 2.0):
        sn = synth.random_state(mesh.n_nodes, 31)
        it = synth.random_state(mesh.n_nodes, 32)
        sn["dv"] *= scale
        it["dv"] *= scale
        K, _, _, _ = NW.linear_system(disc, ti, NW.stage(sn, it, am, af), 0.5)
        A = AS.split_blocks(K.tocsr())[0]
        skew.append(spla.norm(A - A.T) / spla.norm(A))
    assert skew[0] <= 1e-14
    assert skew[1] > 1e-8
    assert skew[2] == pytest.approx(2.0 * skew[1], rel=1e-3, abs=0.0)


def test_simple_preconditioner_inverts_its_closed_form():
    """Section 4.3: P_SIMPLE = L diag(A, S^) U equals [[A, A diag(A)^-1 B], [C, D]];
    the factor-by-factor inverse applied to P_SIMPLE x returns x."""
    import scipy.sparse as sp
    Ks, _ = _scaled_blocks()
    A, B, C, D, _, _ = AS.split_blocks(Ks)
    P = sp.bmat([[A, A @ sp.diags(1.0 / A.diagonal()) @ B], [C, D]]).tocsr()
    x = np.random.default_rng(11).standard_normal(P.shape[0])
    y = KR.simple_preconditioner(A, B, C, D)(P @ x)
    np.testing.assert_allclose(y, x, rtol=1e-9, atol=1e-10 * np.abs(x).max())


def test_simple_is_exact_when_A_is_diagonal():
    """With A replaced by its diagonal, P_SIMPLE is the matrix itself, so
    FGMRES preconditioned by it stops after one iteration; with the real A it
    needs more (the case the nested preconditioner is built for)."""
    import scipy.sparse as sp
    Ks, r = _scaled_blocks()
    A, B, C, D, iv, ip = AS.split_blocks(Ks)
    rp = r[np.concatenate([iv, ip])]
    Ad = sp.diags(A.diagonal()).tocsr()
    Kd = sp.bmat([[Ad, B], [C, D]]).tocsr()
    _, its_d, _ = KR.fgmres(lambda z: Kd @ z, rp, KR.simple_preconditioner(Ad, B, C, D), rtol=1e-10, maxit=50)
    assert its_d == 1
    Kp = sp.bmat([[A, B], [C, D]]).tocsr()
    x, its, _ = KR.fgmres(lambda z: Kp @ z, rp, KR.simple_preconditioner(A, B, C, D), rtol=1e-10, maxit=200)
    assert its > 2
    np.testing.assert_allclose(Kp @ x, rp, rtol=0, atol=1e-9 * np.linalg.norm(rp))


def test_lifted_dirichlet_predictor_reaches_the_preset_solution():
    """The lifted predictor changes the Newton path only: the converged steps
    satisfy the same equations (R = 0 on free dofs, R-bar_k = 0, the prescribed
    motion on Dirichlet dofs), so both forms reach the same state."""
    mesh, mat, ti = synth.tube_case(1, 8, 4, dt=0.05, n_steps=20)
    disc = AS.Discretization(mesh, mat)
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    sa, sb = NW.rest_state(mesh), NW.rest_state(mesh)
    for s in range(3):
        sa, ia = NW.time_step(disc, ti, sa, s * ti.dt, tol_R=1e-12, tol_A=1e-9)
        sb, ib = NW.time_step(disc, ti, sb, s * ti.dt, tol_R=1e-12, tol_A=1e-9, lift=True)
        assert ia["converged"] and ib["converged"]
        g = mesh.dir_vel * (s + 1) * ti.dt
        assert np.abs(sb["u"][vm] - g[vm]).max() <= 1e-14
        assert np.abs(sb["v"][vm] - mesh.dir_vel[vm]).max() == 0.0
        for k in ("u", "p", "v", "du", "dp", "dv"):
            scale = np.abs(sa[k]).max()
            assert np.abs(sa[k] - sb[k]).max() <= 1e-8 * scale, (s, k)


def test_lifted_first_corrector_carries_the_boundary_motion():
    """With the lifted predictor the Dirichlet displacement stays at g(t_n) in
    the predictor and reaches g(t_{n+1}) after the first corrector, through
    Delta u-dot = -R-bar_k / alpha_m; R-bar_k then vanishes everywhere (the
    remark after the block reduction), and the interior has moved with the
    boundary (the right-hand-side term K_{.,u-dot} R-bar_k / alpha_m)."""
    mesh, mat, ti = synth.tube_case(1, 8, 4, dt=0.05, n_steps=20)
    disc = AS.Discretization(mesh, mat)
    am, af, gm = E.genalpha(ti.rho_inf)
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    sn = NW.rest_state(mesh)
    it = NW.predictor(mesh, sn, gm, ti.dt, lift=True)
    assert np.abs(it["u"]).max() == 0.0 and np.abs(it["dv"][vm]).max() == 0.0
    st = NW.stage(sn, it, am, af)
    Rk = st["du"] - st["v"]
    K, rhs, _, _ = NW.linear_system(disc, ti, st, 0.0)
    x = NW.solve_scaled(K, rhs, disc.dof_dir)
    it1, _ = NW.newton_update(disc, ti, it, x, Rk, lift=True)
    g = mesh.dir_vel * ti.dt
    np.testing.assert_allclose(it1["u"][vm], g[vm], rtol=0.0, atol=1e-15)
    st1 = NW.stage(sn, it1, am, af)
    assert np.abs(st1["du"] - st1["v"]).max() <= 1e-14 * np.abs(Rk).max()
    free_top = (~vm[:, 2]) & (mesh.X[:, 2] > 1.0)
    assert np.all(it1["u"][free_top, 2] > 0.0)
    with pytest.raises(ValueError):
        NW.time_step(disc, ti, sn, 0.0, rk_corr=False, lift=True)
