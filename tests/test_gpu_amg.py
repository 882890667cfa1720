"""GPU parity of the A-levels' aggregation multigrid against the oracle's
(oracle/amg.py, pinned in tests/test_oracle_amg.py): one V-cycle on the same
scaled A-block to rounding, and nested solves and time steps preconditioned
by it against sparse LU and the oracle's time steps."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import synth
from oracle import amg as AMG
from oracle import assemble as AS
from oracle import element as E
from oracle import newton as NW
from paper_1809_06350_amd import vms as V

from gpu_helpers import rel_err, upload_K

pytestmark = pytest.mark.gpu

OPTS = dict(max_levels=4, min_coarse=8, degree=2, coarse_degree=8)


def _case(name):
    if name == "cube":
        return synth.cube_case(6, nu=0.499, dt=0.05)
    if name == "tube":
        return synth.tube_case(2, 16, 10, dt=0.05, n_steps=20)
    return synth.strip_case(dims=(12, 6, 3), dt=1e-5, t_ramp=1e-4)


def _problem(mesh, mat):
    prob = V.Problem(mesh, mat, "cuda:0")
    if mesh.fibre is not None:
        prob.set_fibres(*synth.fibre_field(mesh, mesh.meta["fibre_rad"]))
    info = prob.setup_amg(V.amg_opts(**OPTS))
    return prob, info


def _oracle_system(mesh, mat, ti, seed):
    """The oracle's tangent at a seeded state (Dirichlet parts zero), unscaled, and its scaled A-block."""
    disc = AS.Discretization(mesh, mat)
    am, af, gm = E.genalpha(ti.rho_inf)
    scale = {"u": 2e-6, "v": 1e-3, "du": 1e-3} if mesh.name.startswith("strip") else {"u": 1e-3, "p": 1e2}
    sn = synth.random_state(mesh.n_nodes, seed, scale)
    it = synth.random_state(mesh.n_nodes, seed + 1, scale)
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    for st in (sn, it):
        for k in ("u", "v", "du", "dv"):
            st[k][vm] = 0.0
    K_o = disc.tangent(NW.stage(sn, it, am, af), (am, af, gm, ti.dt))
    Kd, _ = AS.apply_dirichlet(K_o, np.zeros(K_o.shape[0]), disc.dof_dir)
    W = AS.scaling(Kd)
    Ks = Kd.multiply(W[:, None]).multiply(W[None, :]).tocsr()
    A, _, _, _, iv, _ = AS.split_blocks(Ks)
    return K_o, A, W[iv].reshape(mesh.n_nodes, 3)


@pytest.mark.parametrize("name", ["cube", "tube", "strip"])
@pytest.mark.parametrize("sym", [0, 1])
def test_vcycle_matches_oracle(name, sym):
    mesh, mat, ti = _case(name)
    prob, info = _problem(mesh, mat)
    K_o, A, Wv = _oracle_system(mesh, mat, ti, 11)
    if sym:
        A = ((A + A.T) * 0.5).tocsr()
    dv = mesh.dir_mask[:, 0:3].astype(bool)
    lev = AMG.build(A, Wv, mesh.X, dv, max_levels=OPTS["max_levels"], min_coarse=OPTS["min_coarse"],
                    graph=AMG.mesh_graph(mesh.tets, mesh.n_nodes))
    print(f"[amg {name} sym={sym}] gpu levels {info['n']} oracle {[L.A.shape[0] // L.blk for L in lev]}", flush=True)
    assert info["n_levels"] == len(lev) >= 2
    K = upload_K(prob, K_o)
    prob.prepare(K, torch.zeros(mesh.n_nodes, 4, dtype=torch.float64, device="cuda:0"))
    r = np.random.default_rng(12).standard_normal((mesh.n_nodes, 3))
    r[dv] = 0.0
    z = prob.amg_apply(K, torch.from_numpy(r).cuda(), sym).cpu().numpy()
    zo = AMG.vcycle(lev, r.ravel(), degree=OPTS["degree"], coarse_degree=OPTS["coarse_degree"])
    err = rel_err(z.ravel(), zo)
    print(f"[amg {name} sym={sym}] V-cycle rel err {err:.2e}", flush=True)
    assert err < 1e-11


@pytest.mark.parametrize("name", ["cube", "tube"])
@pytest.mark.parametrize("precision,a_krylov,sym", [(V.FP64, V.AK_CG, 1), (V.FP64, V.AK_CG, 0),
                                                    (V.FP64, V.AK_GMRES, 0), (V.MIXED, V.AK_CG, 0)])
def test_amg_preconditioned_solve_reaches_lu(name, precision, a_krylov, sym):
    mesh, mat, ti = _case(name)
    prob, info = _problem(mesh, mat)
    K_o, _, _ = _oracle_system(mesh, mat, ti, 21)
    mixed = precision == V.MIXED
    K = upload_K(prob, K_o)
    if mixed:
        K.A32, K.B32 = torch.zeros_like(K.A, dtype=torch.float32), torch.zeros_like(K.B, dtype=torch.float32)
        K.C32, K.D32 = torch.zeros_like(K.C, dtype=torch.float32), torch.zeros_like(K.D, dtype=torch.float32)
    rhs_full = np.random.default_rng(22).standard_normal((mesh.n_nodes, 4))
    R = torch.from_numpy(-rhs_full).cuda()
    rhs = prob.prepare(K, R, None, 1e-15, mixed)
    tol = 1e-5 if mixed else 1e-10
    res = {}
    for a_prec in (V.APC_BJ, V.APC_AMG):
        opts = V.solver_opts(rtol=1e-10, rtol_A=tol, rtol_S=tol, rtol_I=tol * 0.1, precision=precision,
                             a_krylov=a_krylov, cg_symmetrise=sym, a_prec=a_prec, maxit_A=1000, maxit_I=1000)
        x, stats = prob.solve_scaled(K, rhs, opts)
        res[a_prec] = (x.cpu().numpy(), stats)
    Kd, rd = AS.apply_dirichlet(K_o, rhs_full.ravel(), AS.Discretization(mesh, mat).dof_dir)
    W = AS.scaling(Kd)
    Ks = Kd.multiply(W[:, None]).multiply(W[None, :]).tocsc()
    xo = spla.splu(Ks).solve(W * rd)
    xa, sa = res[V.APC_AMG]
    xb, sb = res[V.APC_BJ]
    print(f"[amg solve {name}] bj: outer {sb['n_outer']} A {sb['it_A']} I {sb['it_I']}; "
          f"amg: outer {sa['n_outer']} A {sa['it_A']} I {sa['it_I']}", flush=True)
    assert sa["status"] == 0
    assert np.linalg.norm(xa.ravel() - xo) <= 1e-7 * np.linalg.norm(xo)
    assert sa["it_A"] + sa["it_I"] < sb["it_A"] + sb["it_I"]


@pytest.mark.parametrize("precision", [V.FP64, V.MIXED])
def test_lifted_tube_steps_with_amg_match_oracle(precision):
    """Time steps of the small tube at the full workload's stretch rate and step
    (lifted predictor) with the multigrid on both A-levels, against the oracle."""
    mesh, mat, ti = synth.tube_case(1, 16, 20, dt=0.05, n_steps=20)
    prob, _ = _problem(mesh, mat)
    mixed = precision == V.MIXED
    nopts = V.newton_opts(tol_R=1e-8 if mixed else 1e-10, l_max=15, dir_lift=1)
    if mixed:
        sopts = V.solver_opts(rtol=1e-8, precision=V.MIXED, a_krylov=V.AK_CG, cg_symmetrise=0, a_prec=V.APC_AMG)
    else:
        sopts = V.solver_opts(rtol=1e-10, rtol_A=1e-10, rtol_S=1e-10, rtol_I=1e-12, a_krylov=V.AK_CG,
                              cg_symmetrise=0, a_prec=V.APC_AMG, maxit_I=1000, maxit_A=1000)
    st = prob.new_state()
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    for key in ("v_n", "du_n"):
        a = st[key].cpu().numpy()
        a[vm] = mesh.dir_vel[vm]
        st[key].copy_(torch.from_numpy(a))
    disc = AS.Discretization(mesh, mat)
    so = NW.rest_state(mesh)
    K = None
    for s in range(3):
        stats, K = prob.step(st, V.time_int(ti.dt, ti.rho_inf, s * ti.dt, ti.n_steps * ti.dt), nopts, sopts, K)
        so, info = NW.time_step(disc, ti, so, s * ti.dt, tol_R=nopts.tol_R, l_max=15, lift=True)
        print(f"[amg tube step {s}] gpu newton={stats['n_newton']} A={stats['it_A_total']} I={stats['it_I_total']} "
              f"oracle newton={info['n_newton']}", flush=True)
        assert stats["status"] == 0 and info["converged"]
        if not mixed:
            assert stats["n_newton"] == info["n_newton"]
        prob.roll(st)
    tol = 1e-6 if mixed else 1e-7
    for k in ("u", "p", "v") if mixed else ("u", "p", "v", "du", "dp", "dv"):
        assert rel_err(st[k + "_n"].cpu().numpy(), so[k]) < tol, k


@pytest.mark.parametrize("name,degree,coarse,mid", [("strip", 3, 2, 0), ("tube", 2, 4, 4), ("cube", 4, 2, 0),
                                                     ("cube", 2, 3, 5)])
def test_vcycle_matches_oracle_at_bench_settings(name, degree, coarse, mid):
    """The bench's hierarchy shape (three levels) with the smoothing degrees of its workloads
    (3 on the strip; 2 on the finest level of the tube and 4 below it) and other ones."""
    mesh, mat, ti = _case(name)
    opts = dict(max_levels=3, min_coarse=8, degree=degree, coarse_degree=coarse, mid_degree=mid)
    prob = V.Problem(mesh, mat, "cuda:0")
    if mesh.fibre is not None:
        prob.set_fibres(*synth.fibre_field(mesh, mesh.meta["fibre_rad"]))
    info = prob.setup_amg(V.amg_opts(**opts))
    K_o, A, Wv = _oracle_system(mesh, mat, ti, 21)
    dv = mesh.dir_mask[:, 0:3].astype(bool)
    lev = AMG.build(A, Wv, mesh.X, dv, max_levels=3, min_coarse=8, graph=AMG.mesh_graph(mesh.tets, mesh.n_nodes))
    assert info["n_levels"] == len(lev) >= 2
    assert mid == 0 or len(lev) == 3   # a middle level exists
    K = upload_K(prob, K_o)
    prob.prepare(K, torch.zeros(mesh.n_nodes, 4, dtype=torch.float64, device="cuda:0"))
    r = np.random.default_rng(22).standard_normal((mesh.n_nodes, 3))
    r[dv] = 0.0
    z = prob.amg_apply(K, torch.from_numpy(r).cuda(), 0).cpu().numpy()
    zo = AMG.vcycle(lev, r.ravel(), degree=degree, coarse_degree=coarse, mid_degree=mid)
    err = rel_err(z.ravel(), zo)
    print(f"[amg {name} degree={degree} coarse={coarse} mid={mid}] V-cycle rel err {err:.2e}", flush=True)
    assert err < 1e-11
