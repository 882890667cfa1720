"""Parity at the benchmark sizes, where the oracle cannot solve.

* sampled rows: at a seeded state on the 64^3 cube (the full tube, the
  tensile strip at 1/dx = 400) the
  oracle computes the element residuals/tangents of the elements around a
  few sampled nodes and sums them into those nodes' rows; the GPU rows must
  agree to 1e-11 of the largest entry;
* the converged state of a GPU time step in the benchmark's launch
  configuration satisfies the oracle's own discrete equations: the oracle's
  norm of (R-bar_k, R_p, R_m) at that state, relative to its norm at the
  predictor, is below the Newton tolerance (FP64 and mixed forms; 64^3
  nu = 0.499, the 32^3 Poisson-ratio sweep, the full-size HGO tube, the
  tensile strip at 1/dx = 200);
* the adjoint gradient at 32^3 matches central differences of the GPU
  forward run (h = 1e-6 relative).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import assemble as AS
from oracle import element as E
from oracle import material as M
from oracle import newton as NW
from paper_1809_06350_amd import adjoint as GA
from paper_1809_06350_amd import vms as V

pytestmark = pytest.mark.gpu


def _problem(mesh, mat):
    prob = V.Problem(mesh, mat, "cuda:0")
    if mesh.fibre is not None:
        fib, dfib = synth.fibre_field(mesh, mesh.meta["fibre_rad"])
        prob.set_fibres(fib, dfib)
    return prob


def _sampled_rows(mesh, mat, ti, prob, seed, n_sample=12):
    rng = np.random.default_rng(seed)
    nodes = rng.choice(mesh.n_nodes, n_sample, replace=False)
    # displacements well below the element size (1/64 and 1/80; 12.5 um across the strip's thickness)
    small = {"u": 1e-7, "v": 1e-3, "du": 1e-3} if mesh.name.startswith("strip") else {"u": 1e-4}
    sn = synth.random_state(mesh.n_nodes, seed, small)
    it = synth.random_state(mesh.n_nodes, seed + 1, small)
    st = prob.new_state()
    for k in ("u", "p", "v", "du", "dp", "dv"):
        st[k + "_n"].copy_(torch.from_numpy(sn[k]))
        st[k].copy_(torch.from_numpy(it[k]))
    t_n = 0.3 * ti.dt
    K, R, corr = prob.assemble(st, V.time_int(ti.dt, ti.rho_inf, t_n, ti.n_steps * ti.dt),
                               V.ASM_RESIDUAL | V.ASM_TANGENT | V.ASM_RKCORR)
    torch.cuda.synchronize()
    # oracle on the elements around the sampled nodes
    elems = np.nonzero(np.isin(mesh.tets, nodes).any(axis=1))[0]
    t = mesh.tets[elems]
    Xe = mesh.X[t]
    Vv, G = E.ref_geometry(Xe)
    tau = E.tau_m(Xe, mat)
    H = M.structure_tensors(mesh.fibre[elems], mat.kd) if mesh.fibre is not None else None
    am, af, gm = E.genalpha(ti.rho_inf)
    sto = NW.stage(sn, it, am, af)
    g = {k: sto[k][t] for k in ("dv", "dp", "u", "p", "v")}
    Re = E.element_residual(Vv, G, tau, mat, H, g["dv"], g["dp"], g["u"], g["p"], g["v"])
    Ke = E.element_tangent(Vv, G, tau, mat, H, (am, af, gm, ti.dt), g["dv"], g["dp"], g["u"], g["p"], g["v"])
    Rk = (sto["du"] - sto["v"])[t]
    Je = E.element_u_jvp(Vv, G, tau, mat, H, Rk, g["dv"], g["dp"], g["u"], g["p"], g["v"])
    h = prob.host
    Rg, cg = R.cpu().numpy(), corr.cpu().numpy()
    A, B, C, D = (x.cpu().numpy() for x in (K.A, K.B, K.C, K.D))
    fext = AS.Discretization(mesh, mat).nodal_traction(NW.load_scale(ti, t_n + af * ti.dt))
    for node in nodes:
        row_o = np.zeros(4)
        corr_o = np.zeros(4)
        blocks = {}
        for ei in range(len(elems)):
            for A_ in range(4):
                if t[ei, A_] != node:
                    continue
                row_o += Re[ei, A_]
                corr_o += (af * gm * ti.dt / am) * Je[ei, A_]
                for B_ in range(4):
                    blocks.setdefault(t[ei, B_], np.zeros((4, 4)))
                    blocks[t[ei, B_]] += Ke[ei, A_, :, B_, :]
        row_o[0:3] += fext[node]
        for j, blk_o in blocks.items():
            lo = h["row_ptr"][node]
            hi = lo + h["row_len"][node]
            b = lo + int(np.searchsorted(h["col"][lo:hi], j))
            assert h["col"][b] == j
            yield "A", A[:, b].reshape(3, 3), blk_o[0:3, 0:3]
            yield "B", B[:, b], blk_o[0:3, 3]
            yield "C", C[:, b], blk_o[3, 0:3]
            yield "D", D[b], blk_o[3, 3]
        yield "R_m", Rg[node, 0:3], row_o[0:3]
        yield "R_p", Rg[node, 3], row_o[3]
        yield "corr_m", cg[node, 0:3], corr_o[0:3]
        yield "corr_p", cg[node, 3], corr_o[3]


@pytest.mark.parametrize("name", ["cube64", "tube", "strip400"])
def test_sampled_rows_at_full_size(name):
    if name == "cube64":
        mesh, mat, ti = synth.cube_case(64, nu=0.499, n_steps=10)
    elif name == "strip400":
        mesh, mat, ti = synth.strip_case(400)
    else:
        mesh, mat, ti = synth.tube_case(8, 256, 160, dt=1e-3, n_steps=20, stretch=1.001)
    prob = _problem(mesh, mat)
    scale = {}
    pairs = list(_sampled_rows(mesh, mat, ti, prob, 17))
    for kind, g, o in pairs:
        scale[kind] = max(scale.get(kind, 0.0), np.abs(o).max())
    print(f"[rows] {name} {len(pairs)} sampled arrays", flush=True)
    for kind, g, o in pairs:
        assert np.abs(np.asarray(g) - o).max() <= 1e-11 * scale[kind], kind


def _oracle_residual_ratio(mesh, mat, ti, s, state_n, state_np1):
    """Oracle norm of (R-bar_k, R_p, R_m) at the given iterate over its norm at the predictor."""
    disc = AS.Discretization(mesh, mat)
    am, af, gm = E.genalpha(ti.rho_inf)
    load = NW.load_scale(ti, s * ti.dt + af * ti.dt)

    def norm(it):
        st = NW.stage(state_n, it, am, af)
        return NW.residual_norm(disc, disc.residual(st, load), st["du"] - st["v"])
    pred = NW.predictor(mesh, state_n, gm, (s + 1) * ti.dt)
    return norm(state_np1) / norm(pred)


def _gpu_steps(prob, mesh, ti, n_steps, sopts, tol=1e-8, tol_abs=1e-50, lift=0):
    st = prob.new_state()
    vm = torch.from_numpy(mesh.dir_mask[:, 0:3].astype(bool)).cuda()
    dv = torch.from_numpy(mesh.dir_vel).cuda()
    for key in ("v_n", "du_n"):
        st[key][vm] = dv[vm]
    states = [{k: st[k + "_n"].cpu().numpy().copy() for k in ("u", "p", "v", "du", "dp", "dv")}]
    K = None
    for s in range(n_steps):
        stats, K = prob.step(st, V.time_int(ti.dt, ti.rho_inf, s * ti.dt, ti.n_steps * ti.dt),
                             V.newton_opts(tol_R=tol, tol_A=tol_abs, dir_lift=lift), sopts, K)
        assert stats["status"] == 0
        states.append({k: st[k].cpu().numpy().copy() for k in ("u", "p", "v", "du", "dp", "dv")})
        prob.roll(st)
        print(f"[gpu step {s}] newton={stats['n_newton']} outer={stats['it_outer_total']} A={stats['it_A_total']} "
              f"S={stats['it_S_total']} I={stats['it_I_total']} ms={stats['ms_total']:.1f}", flush=True)
    return states


@pytest.mark.parametrize("precision", [V.FP64, V.MIXED])
def test_cube64_time_step_satisfies_oracle_equations(precision):
    mesh, mat, ti = synth.cube_case(64, nu=0.499, n_steps=10)
    prob = _problem(mesh, mat)
    # the benchmark configuration: GMRES A-levels in FP64, CG on A itself in the mixed form
    ak = V.AK_CG if precision == V.MIXED else V.AK_GMRES
    sopts = V.solver_opts(rtol=1e-8, precision=precision, a_krylov=ak, cg_symmetrise=0)
    states = _gpu_steps(prob, mesh, ti, 1, sopts)
    ratio = _oracle_residual_ratio(mesh, mat, ti, 0, states[0], states[1])
    print(f"[cube64] precision={precision} oracle |R|/|R0| = {ratio:.3e}", flush=True)
    assert ratio <= 1.5e-8


@pytest.mark.parametrize("nu", [0.3, 0.45, 0.499, 0.5])
def test_cube32_poisson_sweep_satisfies_oracle_equations(nu):
    """The 32^3 Poisson-ratio sweep over the full 10-step load ramp (every step must converge);
    the oracle's equations are checked at the first, a middle and the last step."""
    mesh, mat, ti = synth.cube_case(32, nu=nu, n_steps=10)
    prob = _problem(mesh, mat)
    states = _gpu_steps(prob, mesh, ti, 10, V.solver_opts(rtol=1e-8))
    for s in (0, 5, 9):
        ratio = _oracle_residual_ratio(mesh, mat, ti, s, states[s], states[s + 1])
        print(f"[sweep32] nu={nu} step {s} oracle |R|/|R0| = {ratio:.3e}", flush=True)
        assert ratio <= 1.5e-8, (nu, s, ratio)


def _oracle_force_ratio(mesh, mat, ti, s, state_n, state_np1):
    """Oracle norm of (R-bar_k, R_p, R_m) at a converged iterate of the lifted form over the norm
    of the internal force vector there: R_m with every rate and the pressure set to zero (the
    preset predictor of the full tube stretches its end layer five-fold, so its residual is no
    scale for the equations)."""
    disc = AS.Discretization(mesh, mat)
    am, af, gm = E.genalpha(ti.rho_inf)
    load = NW.load_scale(ti, s * ti.dt + af * ti.dt)
    st = NW.stage(state_n, state_np1, am, af)
    num = NW.residual_norm(disc, disc.residual(st, load), st["du"] - st["v"])
    still = {k: np.zeros_like(v) for k, v in st.items()}
    still["u"] = st["u"]
    f_int = disc.residual(still, 0.0)[:, 0:3][~disc.vmask]
    return num / np.linalg.norm(f_int)


def test_full_tube_time_steps_satisfy_oracle_equations():
    """Config 4 at its loading: the full tube (8 x 256 x 160 hexes) stretched at the rate that
    reaches 1.5 in 20 steps of 0.05, lifted predictor, multigrid on the A-levels and the
    pressure-mass Schur preconditioner, mixed form; two steps from rest against the oracle's
    equations (relative to the internal force)."""
    mesh, mat, ti = synth.tube_case(8, 256, 160, dt=0.05, n_steps=20, stretch=1.5)
    prob = _problem(mesh, mat)
    prob.setup_amg(V.amg_opts(coarse_degree=4, mid_degree=4))   # the bench's tube hierarchy
    sopts = V.solver_opts(rtol=1e-8, precision=V.MIXED, a_krylov=V.AK_CG, cg_symmetrise=0, a_prec=V.APC_AMG,
                          schur_mass=1.0, shat_method=V.SHAT_NONE)
    states = _gpu_steps(prob, mesh, ti, 2, sopts, tol_abs=1e-15, lift=1)
    for s in (0, 1):
        ratio = _oracle_force_ratio(mesh, mat, ti, s, states[s], states[s + 1])
        end = states[s + 1]["u"][mesh.dir_mask[:, 2].astype(bool) & (mesh.X[:, 2] > 1.0), 2]
        print(f"[tube] step {s} oracle |R| / |f_int| = {ratio:.3e}, end face u_z = {end.min():.6f}", flush=True)
        assert np.allclose(end, (s + 1) * ti.dt * mesh.dir_vel[mesh.dir_mask[:, 2].astype(bool) & (mesh.X[:, 2] > 1.0), 2])
        assert ratio <= 1e-8


@pytest.mark.parametrize("relax", [0, 1])
@pytest.mark.parametrize("precision", [V.FP64, V.MIXED])
def test_full_strip_time_steps_satisfy_oracle_equations(precision, relax):
    """The eighth-strip at 1/dx = 200 (200 x 60 x 10 hexes, 720,000 tets) at the
    paper's dt = 1e-5, three steps from rest with the bench's options for the
    strip (CG at the A-levels), with and without the relaxed inner tolerance.  The
    first step's initial residual is ~1e-9 against a round-off floor near
    2e-17 (the load is 1e-7 of full), so it ends at the 1e-15 absolute
    tolerance; the next two are checked against the oracle's equations."""
    mesh, mat, ti = synth.strip_case(200)
    prob = _problem(mesh, mat)
    sopts = V.solver_opts(rtol=1e-8, precision=precision, a_krylov=V.AK_CG, cg_symmetrise=0, relax_inner=relax)
    states = _gpu_steps(prob, mesh, ti, 3, sopts, tol_abs=1e-15)
    for s in (1, 2):
        ratio = _oracle_residual_ratio(mesh, mat, ti, s, states[s], states[s + 1])
        print(f"[strip200] precision={precision} relax={relax} step {s} oracle |R|/|R0| = {ratio:.3e}", flush=True)
        assert ratio <= 1.5e-8


@pytest.mark.parametrize("precision", [V.FP64, V.MIXED])
def test_full_strip_time_steps_with_the_bench_options_satisfy_oracle_equations(precision):
    """The same strip with the bench's strip options: CG at the A-levels preconditioned by the
    multigrid (three levels, Chebyshev degree 3), the Schur level by CG steps on S^ plus the
    pressure-mass term."""
    mesh, mat, ti = synth.strip_case(200)
    prob = _problem(mesh, mat)
    prob.setup_amg(V.amg_opts(max_levels=3, degree=3))
    sopts = V.solver_opts(rtol=1e-8, precision=precision, a_krylov=V.AK_CG, cg_symmetrise=0, a_prec=V.APC_AMG,
                          schur_mass=1.0, shat_method=V.SHAT_CG)
    states = _gpu_steps(prob, mesh, ti, 3, sopts, tol_abs=1e-15)
    for s in (1, 2):
        ratio = _oracle_residual_ratio(mesh, mat, ti, s, states[s], states[s + 1])
        print(f"[strip200 multigrid] precision={precision} step {s} oracle |R|/|R0| = {ratio:.3e}", flush=True)
        assert ratio <= 1.5e-8


def _adjoint_vs_fd(mesh, mat, ti, n_steps, sel, params, theta0, seed, sopts, nopts, rel, h_rel=None, amg=False):
    """J = 1/2 ||u_sel - u_target||^2 with u_target from a forward run at seeded, perturbed
    parameters; the autograd gradient against central differences (step h_rel[k] relative,
    1e-6 by default, tolerance rel[k] relative with no absolute floor)."""
    h_rel = h_rel or {}
    prob = _problem(mesh, mat)
    if amg:
        prob.setup_amg()
    pmask = sum(1 << k for k in params)
    hist = GA.TimeHistory(prob, ti, n_steps, nopts, sopts, sopts, pmask)
    rng = np.random.default_rng(seed)
    th_t = theta0.copy()
    for k in params:
        th_t[k] *= 1.0 + 0.05 * rng.uniform(-1.0, 1.0)
    selt = torch.from_numpy(sel).cuda()
    target = hist.run(th_t)[selt].clone()

    def J_of(theta):
        u = hist.run(theta)
        print("[adjoint] forward Newton histories:", [st["res_norm"] for st in hist.stats], flush=True)
        return 0.5 * float(((u[selt] - target) ** 2).sum())

    theta = torch.tensor(theta0, requires_grad=True)
    u = GA.VmsAdjoint.apply(theta, hist)
    J = 0.5 * ((u[selt] - target) ** 2).sum()
    J.backward()
    g = theta.grad.numpy()
    for k in params:
        h = h_rel.get(k, 1e-6) * abs(theta0[k])
        tp, tm = theta0.copy(), theta0.copy()
        tp[k] += h
        tm[k] -= h
        fd = (J_of(tp) - J_of(tm)) / (2 * h)
        print(f"[adjoint] param {k}: adjoint={g[k]:.10e} fd={fd:.10e} rel.diff={abs(g[k] - fd) / abs(fd):.2e}",
              flush=True)
        assert g[k] == pytest.approx(fd, rel=rel[k], abs=0.0)


def test_cube32_adjoint_matches_central_differences():
    mesh, mat, ti = synth.cube_case(32, nu=0.499, n_steps=10)
    sopts = V.solver_opts(rtol=1e-12, rtol_A=1e-12, rtol_S=1e-12, rtol_I=1e-13)
    theta0 = np.array([mat.mu, mat.kappa, 0.0, 0.0, 0.0])
    _adjoint_vs_fd(mesh, mat, ti, 2, np.isclose(mesh.X[:, 2], 1.0), (0, 1), theta0, 5, sopts,
                   V.newton_opts(tol_R=1e-12), rel={0: 1e-5, 1: 1e-5})


def test_tube_adjoint_matches_central_differences():
    """The artery mesh at an eighth of the full size (4 x 128 x 80 hexes, 245 760 tets; a tight
    FP64 forward step of the full mesh takes about 40 s, and central differences need nine) at
    the full workload's loading (one step of 0.05 towards the stretch 1.5, lifted predictor):
    dJ/d(mu, k1, k2, fibre angle) by the adjoint against central differences with the relative
    step 1e-6 of config 5 in every parameter.  FP64 forward and adjoint solves, multigrid on the
    A-levels and the pressure-mass Schur preconditioner."""
    mesh, mat, ti = synth.tube_case(4, 128, 80, dt=0.05, n_steps=20, stretch=1.5)
    sopts = V.solver_opts(rtol=1e-12, rtol_A=1e-11, rtol_S=1e-11, rtol_I=1e-12, a_krylov=V.AK_CG, cg_symmetrise=0,
                          a_prec=V.APC_AMG, schur_mass=1.0, shat_method=V.SHAT_NONE, maxit_A=1000, maxit_I=1000)
    theta0 = np.array([mat.mu, 0.0, mat.k1, mat.k2, mesh.meta["fibre_rad"]])
    r = np.hypot(mesh.X[:, 0], mesh.X[:, 1])
    _adjoint_vs_fd(mesh, mat, ti, 1, np.isclose(r, 1.2), (0, 2, 3, 4), theta0, 6, sopts,
                   V.newton_opts(tol_R=1e-11, tol_A=1e-15, l_max=30, dir_lift=1),
                   rel={0: 1e-5, 2: 1e-5, 3: 1e-5, 4: 1e-5}, amg=True)
