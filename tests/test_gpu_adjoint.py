"""GPU parity of the adjoint path against the oracle's adjoint (which is
itself pinned by central differences of the forward run)."""
import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as AD
from oracle import assemble as AS
from oracle import element as E
from oracle import newton as NW
from paper_1809_06350_amd import adjoint as GA
from paper_1809_06350_amd import vms as V

from gpu_helpers import gpu_K_scipy, rel_err

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "cube":
        mesh, mat, ti = synth.cube_case(3, nu=0.45, n_steps=2)
        return mesh, mat, ti, 0b00011, np.isclose(mesh.X[:, 2], 1.0)
    if name == "tube":
        mesh, mat, ti = synth.tube_case(1, 8, 2, dt=0.05, n_steps=20)
        r = np.hypot(mesh.X[:, 0], mesh.X[:, 1])
        return mesh, mat, ti, 0b11101, np.isclose(r, 1.2)
    # the eighth-strip (in-plane fibres, dispersion), load ramped over 0.1 ms
    mesh, mat, ti = synth.strip_case(dims=(5, 3, 2), dt=1e-5, t_ramp=1e-4)
    return mesh, mat, ti, 0b11101, np.isclose(mesh.X[:, 0], 5e-3, rtol=0.0, atol=1e-12)


def _prob(mesh, mat):
    prob = V.Problem(mesh, mat, "cuda:0")
    if mesh.fibre is not None:
        fib, dfib = synth.fibre_field(mesh, mesh.meta["fibre_rad"])
        prob.set_fibres(fib, dfib)
    return prob


def _consistent_states(mesh, ti, seed):
    """(s_n, s_{n+1}) with y_{n+1} from the generalized-alpha update, Dirichlet parts zero."""
    am, af, gm = E.genalpha(ti.rho_inf)
    # the strip's elements are 0.1-1 mm across: displacements and rates at that scale
    scale = {"u": 2e-6, "v": 1e-3, "du": 1e-3} if mesh.name.startswith("strip") else None
    sn = synth.random_state(mesh.n_nodes, seed, scale)
    s1 = synth.random_state(mesh.n_nodes, seed + 1, scale)
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    for st in (sn, s1):
        for k in ("u", "v", "du", "dv"):
            st[k][vm] = 0.0
    for v, r in (("u", "du"), ("p", "dp"), ("v", "dv")):
        s1[v] = sn[v] + ti.dt * sn[r] + gm * ti.dt * (s1[r] - sn[r])
    return sn, s1


def _gpu_state(prob, sn, s1):
    st = prob.new_state()
    for k in ("u", "p", "v", "du", "dp", "dv"):
        st[k + "_n"].copy_(torch.from_numpy(sn[k]))
        st[k].copy_(torch.from_numpy(s1[k]))
    return st


@pytest.mark.parametrize("name,a_krylov", [("cube", 0), ("tube", 0), ("cube", 2), ("strip", 2)])
def test_transposed_solve_matches_oracle(name, a_krylov):
    mesh, mat, ti, pmask, sel = _case(name)
    prob = _prob(mesh, mat)
    sn, s1 = _consistent_states(mesh, ti, 5)
    st = _gpu_state(prob, sn, s1)
    tiv = V.time_int(ti.dt, ti.rho_inf, 0.0, ti.n_steps * ti.dt)
    K, R, _ = prob.assemble(st, tiv, V.ASM_RESIDUAL | V.ASM_TANGENT)
    prob.prepare(K, R)
    am, af, gm = E.genalpha(ti.rho_inf)
    disc = AS.Discretization(mesh, mat)
    Ko = disc.tangent(NW.stage(sn, s1, am, af), (am, af, gm, ti.dt))
    Kd, _ = AS.apply_dirichlet(Ko, np.zeros(Ko.shape[0]), disc.dof_dir)
    W = AS.scaling(Kd)
    Ks = Kd.multiply(W[:, None]).multiply(W[None, :]).tocsr()
    rhs = np.random.default_rng(2).standard_normal(4 * mesh.n_nodes)
    rhs[disc.dof_dir] = 0.0
    Kt = prob.new_matrix()
    opts = V.solver_opts(rtol=1e-11, rtol_A=1e-12, rtol_S=1e-12, rtol_I=1e-13, a_krylov=a_krylov, cg_symmetrise=0)
    lam, stats = prob.solve_transpose_scaled(K, Kt, torch.from_numpy(rhs.reshape(-1, 4)).cuda(), opts)
    lg = lam.cpu().numpy().ravel()
    print(f"[transpose] {name} {stats}", flush=True)
    # lambda solves the transposed system of the GPU's scaled matrix, which is the
    # oracle's up to the rounding of assembly
    Kg = gpu_K_scipy(prob, K)
    assert abs(Kg - Ks).max() <= 1e-11 * abs(Ks).max()
    # residual to 1e-10 of the right-hand side, above the rounding floor of evaluating K^T lambda
    # (1e-13 of |K^T| |lambda|: the strip's system at dt = 1e-5 is ill-conditioned and lambda large)
    floor = 1e-13 * np.linalg.norm(abs(Kg).T @ np.abs(lg))
    print(f"[transpose] {name} |lambda| = {np.linalg.norm(lg):.3e} floor = {floor:.3e}", flush=True)
    assert np.linalg.norm(Kg.T @ lg - rhs) <= 1e-10 * np.linalg.norm(rhs) + floor
    assert np.linalg.norm(Ks.T @ lg - rhs) <= 1e-10 * np.linalg.norm(rhs) + floor + 1e-11 * np.linalg.norm(
        abs(Ks).T @ np.abs(lg))


@pytest.mark.parametrize("name,precision", [("cube", V.FP64), ("tube", V.FP64), ("cube", V.MIXED)])
def test_unscaled_transposed_solve_matches_lu(name, precision):
    """vms_solve_transpose: K as assembled in, K^T lam = g out (Dirichlet rows and
    columns of K replaced by the identity, lam = 0 there), against sparse LU on
    the oracle's K^T."""
    import scipy.sparse.linalg as spla
    mesh, mat, ti, pmask, sel = _case(name)
    prob = _prob(mesh, mat)
    sn, s1 = _consistent_states(mesh, ti, 6)
    st = _gpu_state(prob, sn, s1)
    tiv = V.time_int(ti.dt, ti.rho_inf, 0.0, ti.n_steps * ti.dt)
    mixed = precision == V.MIXED
    K, _, _ = prob.assemble(st, tiv, V.ASM_TANGENT)
    if mixed:
        K2 = prob.new_matrix(mirror32=True)
        for a, b in ((K2.A, K.A), (K2.B, K.B), (K2.C, K.C), (K2.D, K.D)):
            a.copy_(b)
        K = K2
    am, af, gm = E.genalpha(ti.rho_inf)
    disc = AS.Discretization(mesh, mat)
    Ko = disc.tangent(NW.stage(sn, s1, am, af), (am, af, gm, ti.dt))
    Kd, _ = AS.apply_dirichlet(Ko, np.zeros(Ko.shape[0]), disc.dof_dir)
    g = np.random.default_rng(3).standard_normal(4 * mesh.n_nodes)
    opts = (V.solver_opts(rtol=1e-11, rtol_A=1e-6, rtol_S=1e-6, rtol_I=1e-6, precision=V.MIXED, maxit=400)
            if mixed else V.solver_opts(rtol=1e-11, rtol_A=1e-12, rtol_S=1e-12, rtol_I=1e-13))
    Kt = prob.new_matrix(mirror32=mixed)
    lam, stats = prob.solve_transpose(K, Kt, torch.from_numpy(g.reshape(-1, 4)).cuda(), opts)
    lg = lam.cpu().numpy().ravel()
    gd = np.where(disc.dof_dir, 0.0, g)
    lo = spla.splu(Kd.T.tocsc()).solve(gd)
    print(f"[transpose unscaled] {name} precision={precision} {stats}", flush=True)
    assert stats["status"] == 0 and stats["phases_timed"] == 1
    assert np.all(lg[disc.dof_dir] == 0.0)
    W = AS.scaling(Kd)
    assert rel_err(K.W.cpu().numpy().ravel(), W) < 1e-13
    # residual of the scaled transposed system (W K^T W) lam* = W g, lam* = lam / W
    Ks = Kd.multiply(W[:, None]).multiply(W[None, :]).tocsr()
    assert np.linalg.norm(Ks.T @ (lg / W) - W * gd) <= 1e-10 * np.linalg.norm(W * gd)
    assert np.linalg.norm(lg - lo) <= 1e-7 * np.linalg.norm(lo)


@pytest.mark.parametrize("name", ["cube", "tube", "strip"])
def test_parameter_sensitivities_match_oracle(name):
    mesh, mat, ti, pmask, sel = _case(name)
    prob = _prob(mesh, mat)
    sn, s1 = _consistent_states(mesh, ti, 7)
    st = _gpu_state(prob, sn, s1)
    lam = np.random.default_rng(4).standard_normal((mesh.n_nodes, 4))
    tiv = V.time_int(ti.dt, ti.rho_inf, 0.0, ti.n_steps * ti.dt)
    g = prob.param_sensitivity(st, tiv, torch.from_numpy(lam).cuda(), pmask)
    theta = AD.theta_of(mesh, mat)
    lam7 = np.zeros((mesh.n_nodes, 7))
    lam7[:, 3] = lam[:, 3]
    lam7[:, 4:7] = lam[:, 0:3]
    for k in range(5):
        if pmask & (1 << k):
            o = AD.theta_cotangent(mesh, mat, ti, theta, sn, s1, lam7, k)
            print(f"[sens] {name} {AD.PARAMS[k]} gpu={g[k]:.12e} oracle={o:.12e}", flush=True)
            assert g[k] == pytest.approx(o, rel=1e-9, abs=1e-14 * abs(o) + 1e-300)


@pytest.mark.parametrize("name", ["cube", "tube", "strip"])
def test_backward_step_matches_oracle(name):
    mesh, mat, ti, pmask, sel = _case(name)
    prob = _prob(mesh, mat)
    states = AD.forward(mesh, mat, ti, 1)
    sn, s1 = states
    st = _gpu_state(prob, sn, s1)
    rng = np.random.default_rng(9)
    ybar = rng.standard_normal((mesh.n_nodes, 7))
    ydbar = rng.standard_normal((mesh.n_nodes, 7)) * 1e-3
    theta = AD.theta_of(mesh, mat)
    params = tuple(k for k in range(5) if pmask & (1 << k))
    yb0, ydb0, dth, _ = AD.backward_step(mesh, mat, ti, theta, sn, s1, ybar, ydbar, params)
    K = prob.new_matrix()
    Kt = prob.new_matrix()
    dJ = np.zeros(5)
    opts = V.solver_opts(rtol=1e-12, rtol_A=1e-12, rtol_S=1e-12, rtol_I=1e-13)
    gyb, gydb, stats = prob.adjoint_step(st, V.time_int(ti.dt, ti.rho_inf, 0.0, ti.n_steps * ti.dt), K, Kt,
                                         torch.from_numpy(ybar).cuda(), torch.from_numpy(ydbar).cuda(), pmask,
                                         dJ, opts)
    print(f"[backward] {name} stats={stats} gpu={dJ} oracle={dth}", flush=True)
    vm = mesh.dir_mask.astype(bool)
    free7 = np.concatenate([~vm[:, 0:3], ~vm[:, 3:4], ~vm[:, 0:3]], axis=1)
    assert rel_err(gyb.cpu().numpy()[free7], yb0[free7]) < 1e-8
    assert rel_err(gydb.cpu().numpy()[free7], ydb0[free7]) < 1e-8
    for k in params:
        assert dJ[k] == pytest.approx(dth[k], rel=1e-8, abs=1e-12 * np.abs(dth).max())


@pytest.mark.parametrize("name", ["cube", "tube", "strip"])
@pytest.mark.parametrize("precision", [V.FP64, V.MIXED])
def test_autograd_gradient_matches_oracle(name, precision):
    mesh, mat, ti, pmask, sel = _case(name)
    prob = _prob(mesh, mat)
    n_steps = 2
    sopts = V.solver_opts(rtol=1e-12, rtol_A=1e-12, rtol_S=1e-12, rtol_I=1e-13)
    aopts = sopts if precision == V.FP64 else V.solver_opts(rtol=1e-12, rtol_A=1e-5, rtol_S=1e-5, rtol_I=1e-3,
                                                           precision=V.MIXED)
    hist = GA.TimeHistory(prob, ti, n_steps, V.newton_opts(tol_R=1e-12), sopts, aopts, pmask)
    theta0 = AD.theta_of(mesh, mat)
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    u = GA.VmsAdjoint.apply(theta, hist)
    states = AD.forward(mesh, mat, ti, n_steps)
    uo = states[-1]["u"]
    target = torch.from_numpy(uo[sel] * 0.9).cuda()
    selt = torch.from_numpy(sel).cuda()
    J = 0.5 * ((u[selt] - target) ** 2).sum()
    J.backward()
    _, dJo = AD.objective(uo, sel, uo[sel] * 0.9)
    params = tuple(k for k in range(5) if pmask & (1 << k))
    go = AD.adjoint_gradient(mesh, mat, ti, theta0, states, dJo, params)
    gg = theta.grad.numpy()
    print(f"[autograd] {name} precision={precision} gpu={gg} oracle={go}", flush=True)
    assert rel_err(u.detach().cpu().numpy(), uo) < 1e-9
    for k in params:
        assert gg[k] == pytest.approx(go[k], rel=1e-5, abs=0.0), AD.PARAMS[k]


def test_backward_after_a_second_forward_uses_its_own_theta():
    """Two graphs through one TimeHistory at different theta: the first graph's
    backward, run after the second forward, must still give the gradient at the
    first theta and trajectory (against the oracle's adjoint gradient there),
    and the gradient comes back on theta's device."""
    mesh, mat, ti, pmask, sel = _case("cube")
    prob = _prob(mesh, mat)
    sopts = V.solver_opts(rtol=1e-12, rtol_A=1e-12, rtol_S=1e-12, rtol_I=1e-13)
    hist = GA.TimeHistory(prob, ti, 2, V.newton_opts(tol_R=1e-12), sopts, sopts, pmask)
    theta0 = AD.theta_of(mesh, mat)
    states = AD.forward(mesh, mat, ti, 2)
    uo = states[-1]["u"]
    selt = torch.from_numpy(sel).cuda()
    target = torch.from_numpy(uo[sel] * 0.9).cuda()
    t1 = torch.tensor(theta0, dtype=torch.float64, device="cuda:0", requires_grad=True)
    u1 = GA.VmsAdjoint.apply(t1, hist)
    J1 = 0.5 * ((u1[selt] - target) ** 2).sum()
    th2 = theta0.copy()
    th2[0] *= 1.3
    th2[1] *= 0.7
    t2 = torch.tensor(th2, dtype=torch.float64, device="cuda:0", requires_grad=True)
    u2 = GA.VmsAdjoint.apply(t2, hist)
    J2 = 0.5 * ((u2[selt] - target) ** 2).sum()
    J1.backward()
    _, dJo = AD.objective(uo, sel, uo[sel] * 0.9)
    params = tuple(k for k in range(5) if pmask & (1 << k))
    go = AD.adjoint_gradient(mesh, mat, ti, theta0, states, dJo, params)
    assert t1.grad.device == t1.device
    g1 = t1.grad.cpu().numpy()
    print(f"[two graphs] first graph's gradient {g1} oracle {go}", flush=True)
    for k in params:
        assert g1[k] == pytest.approx(go[k], rel=1e-5, abs=0.0)
    # the second graph's gradient is the oracle's at its own theta and trajectory
    J2.backward()
    mesh2, mat2 = AD.with_params(mesh, mat, th2)
    states2 = AD.forward(mesh2, mat2, ti, 2)
    _, dJo2 = AD.objective(states2[-1]["u"], sel, uo[sel] * 0.9)
    go2 = AD.adjoint_gradient(mesh2, mat2, ti, th2, states2, dJo2, params)
    g2 = t2.grad.cpu().numpy()
    print(f"[two graphs] second graph's gradient {g2} oracle {go2}", flush=True)
    for k in params:
        assert g2[k] == pytest.approx(go2[k], rel=1e-5, abs=0.0)
        assert abs(go2[k] - go[k]) > 1e-3 * abs(go[k])
