"""Edge cases and error paths of the C ABI on the GPU: inverted elements,
non-finite states, iteration limits, zero right-hand sides, refused options
and workspaces, nodes outside every element and meshes without elements."""
import ctypes as C
import dataclasses

import numpy as np
import pytest
import torch

import synth
from paper_1809_06350_amd import _lib as L
from paper_1809_06350_amd import vms as V

pytestmark = pytest.mark.gpu


def _ti(ti, t_n=0.0):
    return V.time_int(ti.dt, ti.rho_inf, t_n, ti.n_steps * ti.dt)


def _system(N=3, seed=3):
    """A scaled Newton system of the small cube at a seeded state."""
    mesh, mat, ti = synth.cube_case(N, nu=0.45, n_steps=2)
    prob = V.Problem(mesh, mat, "cuda:0")
    st = prob.new_state()
    rs = synth.random_state(mesh.n_nodes, seed, {"u": 1e-3})
    for k in ("u", "p", "v", "du", "dp", "dv"):
        st[k].copy_(torch.from_numpy(rs[k]))
    K, R, corr = prob.assemble(st, _ti(ti), V.ASM_RESIDUAL | V.ASM_TANGENT | V.ASM_RKCORR)
    rhs = prob.prepare(K, R, corr)
    return prob, mesh, ti, st, K, rhs


def test_inverted_element_is_reported_and_context_survives():
    mesh, mat, ti = synth.cube_case(3, n_steps=2)
    prob = V.Problem(mesh, mat, "cuda:0")
    st = prob.new_state()
    i = int(np.argmin(np.linalg.norm(mesh.X - 1.0 / 3.0, axis=1)))   # an interior node
    st["u"][i] = torch.tensor([3.0, 3.0, 3.0], dtype=torch.float64)
    with pytest.raises(V.VmsError) as ei:
        prob.assemble(st, _ti(ti), V.ASM_RESIDUAL | V.ASM_TANGENT)
    assert ei.value.code == -4
    st["u"].zero_()
    K, R, _ = prob.assemble(st, _ti(ti), V.ASM_RESIDUAL | V.ASM_TANGENT)
    assert torch.isfinite(R).all() and torch.isfinite(K.A).all()


def test_non_finite_state_gives_nan_status():
    mesh, mat, ti = synth.cube_case(3, n_steps=2)
    prob = V.Problem(mesh, mat, "cuda:0")
    st = prob.new_state()
    st["p"][5] = float("nan")
    _, R, _ = prob.assemble(st, _ti(ti), V.ASM_RESIDUAL)
    with pytest.raises(V.VmsError) as ei:
        prob.residual_norm(st, _ti(ti), R)
    assert ei.value.code == -6


def test_iteration_limit_and_zero_rhs():
    prob, mesh, ti, st, K, rhs = _system()
    x, stats = prob.solve_scaled(K, rhs, V.solver_opts(maxit=1), allow_nc=True)
    assert stats["status"] == 1 and stats["n_outer"] == 1
    assert torch.isfinite(x).all() and stats["res"] < stats["res0"]
    z = torch.zeros_like(rhs)
    x0, stats0 = prob.solve_scaled(K, z, V.solver_opts())
    assert stats0["status"] == 0 and stats0["n_outer"] == 0
    assert float(x0.abs().max()) == 0.0


@pytest.mark.parametrize("kw", [dict(maxit=0), dict(maxit_A=1001), dict(maxit_I=0), dict(orth=7),
                                dict(shat_degree=65), dict(precision=2), dict(precond=9), dict(a_krylov=3),
                                dict(a_krylov=V.AK_CG, cg_symmetrise=2), dict(precond=5), dict(schur_solve=2),
                                dict(shat_method=3), dict(relax_inner=2), dict(schur_mass=-1.0),
                                dict(shat_method=V.SHAT_NONE), dict(schur_mass=1.0, precond=V.PC_SIMPLE),
                                dict(schur_mass=1.0, schur_solve=V.SCHUR_SHAT)])
def test_bad_solver_options_are_refused(kw):
    prob, mesh, ti, st, K, rhs = _system()
    with pytest.raises(V.VmsError) as ei:
        prob.solve_scaled(K, rhs, V.solver_opts(**kw))
    assert ei.value.code == -1


@pytest.mark.parametrize("sym", [0, 1])
def test_cg_levels_zero_velocity_rhs_and_maxit(sym):
    """CG A-levels: a zero right-hand side (the first A-solve of Algorithm 1
    when the velocity residual vanishes) returns x = 0 at once, and A-levels
    capped at two iterations still give a usable preconditioner (the outer
    FGMRES converges, with more iterations)."""
    prob, mesh, ti, st, K, rhs = _system()
    b = rhs.clone()
    b.view(-1, 4)[:, :3] = 0.0
    for kw in (dict(), dict(maxit_A=2, maxit_I=2)):
        opts = V.solver_opts(a_krylov=V.AK_CG, cg_symmetrise=sym, **kw)
        x, stats = prob.solve_scaled(K, b, opts)
        r = prob.spmv(K, V.OP_FULL, x).reshape(-1) - b.reshape(-1)
        print(f"[cg edge] sym={sym} {kw} stats={stats}", flush=True)
        assert stats["status"] == 0
        assert float(r.norm()) <= 1e-8 * float(b.norm())
        if kw:
            assert stats["it_A"] <= 2 * stats["n_A_solves"] and stats["it_I"] <= 2 * stats["n_I_solves"]


def test_small_workspaces_are_refused():
    prob, mesh, ti, st, K, rhs = _system()
    lib = prob.lib
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda:0")
    x = torch.empty_like(rhs)
    stats = L.SolveStats()
    rc = lib.vms_solve_scaled(prob.ctx, C.byref(prob.cmesh), C.byref(K.c()), rhs.data_ptr(), x.data_ptr(),
                              C.byref(V.solver_opts()), ws.data_ptr(), ws.numel(), C.byref(stats))
    assert rc == -3
    R = torch.empty(mesh.n_nodes, 4, dtype=torch.float64, device="cuda:0")
    # the residual alone goes through element vectors (128 B per element)
    assert lib.vms_assemble_workspace(C.byref(prob.cmesh), V.ASM_RESIDUAL) > ws.numel()
    rc = lib.vms_assemble(prob.ctx, C.byref(prob.cmesh), C.byref(prob.cmat), C.byref(_ti(ti)),
                          C.byref(prob.cstate(st)), prob.f_ext.data_ptr(), None, R.data_ptr(), None,
                          V.ASM_RESIDUAL, ws.data_ptr(), ws.numel())
    assert rc == -3
    # the tangent on 16-slot rows is assembled by the row owners and needs 1 KB only
    assert lib.vms_assemble_workspace(C.byref(prob.cmesh), V.ASM_RESIDUAL | V.ASM_TANGENT) == 1024
    rc = lib.vms_assemble(prob.ctx, C.byref(prob.cmesh), C.byref(prob.cmat), C.byref(_ti(ti)),
                          C.byref(prob.cstate(st)), prob.f_ext.data_ptr(), C.byref(K.c()), R.data_ptr(), None,
                          V.ASM_RESIDUAL | V.ASM_TANGENT, ws.data_ptr(), 512)
    assert rc == -3
    rc = lib.vms_assemble(prob.ctx, C.byref(prob.cmesh), C.byref(prob.cmat), C.byref(_ti(ti)),
                          C.byref(prob.cstate(st)), prob.f_ext.data_ptr(), C.byref(K.c()), R.data_ptr(), None,
                          V.ASM_RESIDUAL | V.ASM_TANGENT, ws.data_ptr(), ws.numel())
    assert rc == 0
    rc = lib.vms_assemble(prob.ctx, C.byref(prob.cmesh), C.byref(prob.cmat), C.byref(_ti(ti)),
                          C.byref(prob.cstate(st)), prob.f_ext.data_ptr(), C.byref(K.c()), R.data_ptr(), None,
                          0, ws.data_ptr(), ws.numel())
    assert rc == -1


def test_isolated_nodes_change_nothing_else():
    """Two nodes outside every element: their rows are zero (no load on them) and every other
    assembled value is bitwise the same as without them."""
    mesh, mat, ti = synth.cube_case(3, nu=0.45, n_steps=2)
    n0 = mesh.n_nodes
    m2 = dataclasses.replace(mesh, X=np.vstack([mesh.X, [[5.0, 5.0, 5.0], [6.0, 6.0, 6.0]]]),
                             dir_mask=np.vstack([mesh.dir_mask, np.zeros((2, 4), np.uint8)]),
                             dir_vel=np.vstack([mesh.dir_vel, np.zeros((2, 3))]))
    outs = []
    for mm in (mesh, m2):
        prob = V.Problem(mm, mat, "cuda:0")
        st = prob.new_state()
        rs = synth.random_state(n0, 11, {"u": 1e-3})
        for k in ("u", "p", "v", "du", "dp", "dv"):
            st[k][:n0].copy_(torch.from_numpy(rs[k]))
        K, R, corr = prob.assemble(st, _ti(ti, 0.3 * ti.dt), V.ASM_RESIDUAL | V.ASM_TANGENT | V.ASM_RKCORR)
        W = prob.slot_width
        outs.append((R.cpu().numpy(), corr.cpu().numpy(), K.A.cpu().numpy().reshape(9, -1, W)))
    (R0, c0, A0), (R1, c1, A1) = outs
    assert np.array_equal(R1[:n0], R0) and np.array_equal(c1[:n0], c0)
    assert np.array_equal(A1[:, :n0], A0)
    assert not R1[n0:].any() and not c1[n0:].any() and not A1[:, n0:].any()


def test_mesh_without_elements():
    X = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    mesh = synth.mesh.Mesh("points", X, np.zeros((0, 4), np.int32), np.zeros((0, 3), np.int32),
                           np.zeros((0, 3)), np.zeros((3, 4), np.uint8), np.zeros((3, 3)))
    mat = synth.material_from_nu(1e5, 0.3)
    prob = V.Problem(mesh, mat, "cuda:0")
    st = prob.new_state()
    K, R, corr = prob.assemble(st, V.time_int(1e-3), V.ASM_RESIDUAL | V.ASM_TANGENT | V.ASM_RKCORR)
    torch.cuda.synchronize()
    assert not R.any() and not corr.any()
    assert not K.A.any() and not K.B.any() and not K.C.any() and not K.D.any()
