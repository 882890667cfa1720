"""GPU parity: every step of the HIP Newton step against the CPU FP64 oracle.

Tolerances (FP64 path): block products and assembled arrays agree with the
oracle to 1e-11 of the largest entry of the same array (only the order of
floating-point operations differs: closed-form tangent vs complex step, FMA
contraction, colour-ordered sums); solves reach the requested relative
residual of the oracle's own scaled matrix; a full time step matches the
oracle's displacement to 1e-7 relative (Newton and FGMRES at 1e-10).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import assemble as AS
from oracle import element as E
from oracle import newton as NW
from paper_1809_06350_amd import vms as V

from gpu_helpers import gpu_K_scipy, rel_err, upload_K

pytestmark = pytest.mark.gpu

TOL_ASM = 1e-11


def case(name):
    if name == "cube-comp":
        mesh, mat, ti = synth.cube_case(4, n_steps=2)
    elif name == "cube-incomp":
        mesh, mat, ti = synth.cube_case(3, nu=0.5, n_steps=2)
    elif name == "cube-nu0499":
        mesh, mat, ti = synth.cube_case(5, nu=0.499, n_steps=2)
    elif name == "tube-hgo":
        mesh, mat, ti = synth.tube_case(2, 12, 4, dt=0.05, n_steps=20)
    elif name == "strip-hgo":
        mesh, mat, ti = STRIP()
    elif name == "cube-fan":   # a 32-slot pattern (the fan's centre has 19 blocks in its row)
        mesh, mat, ti = _asm_case_with_fan(True)
    else:
        raise KeyError(name)
    return mesh, mat, ti


def STRIP():
    """A small eighth-strip (10 x 4 x 3 hexes, dispersion 0.226) whose load
    ramps over 1 ms, so that the first steps at the paper's dt = 1e-5 carry a
    load well above round-off."""
    return synth.strip_case(dims=(10, 4, 3), dt=1e-5, t_ramp=1e-3)


# random states at the strip's scale: its elements are 0.08-0.5 mm across
STRIP_STATE = {"u": 2e-6, "v": 1e-3, "du": 1e-3}


def gpu_ti(ti, t_n):
    return V.time_int(ti.dt, ti.rho_inf, t_n, ti.n_steps * ti.dt)


def states(mesh, seed):
    scale = STRIP_STATE if mesh.name.startswith("strip") else None
    sn = synth.random_state(mesh.n_nodes, seed, scale)
    it = synth.random_state(mesh.n_nodes, seed + 1, scale)
    return sn, it


def gpu_state(prob, sn, it):
    st = prob.new_state()
    for k in ("u", "p", "v", "du", "dp", "dv"):
        st[k + "_n"].copy_(torch.from_numpy(sn[k]))
        st[k].copy_(torch.from_numpy(it[k]))
    return st


@pytest.fixture(scope="module")
def problems():
    cache = {}

    def get(name):
        if name not in cache:
            mesh, mat, ti = case(name)
            cache[name] = (V.Problem(mesh, mat, "cuda:0"), mesh, mat, ti, AS.Discretization(mesh, mat))
        return cache[name]
    return get


@pytest.mark.parametrize("name", ["cube-comp", "cube-incomp", "cube-nu0499", "tube-hgo", "strip-hgo"])
def test_assembly_matches_oracle(problems, name):
    prob, mesh, mat, ti, disc = problems(name)
    print(f"[assembly] {name} n={mesh.n_nodes} m={mesh.n_tets}", flush=True)
    sn, it = states(mesh, 31)
    t_n = 0.4 * ti.dt
    st = gpu_state(prob, sn, it)
    K, R, corr = prob.assemble(st, gpu_ti(ti, t_n), V.ASM_RESIDUAL | V.ASM_TANGENT | V.ASM_RKCORR)
    torch.cuda.synchronize()
    am, af, gm = E.genalpha(ti.rho_inf)
    sto = NW.stage(sn, it, am, af)
    load = NW.load_scale(ti, t_n + af * ti.dt)
    R_o = disc.residual(sto, load)
    K_o = disc.tangent(sto, (am, af, gm, ti.dt))
    corr_o = (af * gm * ti.dt / am) * disc.u_jvp(sto, sto["du"] - sto["v"])
    Rg = R.cpu().numpy()
    assert rel_err(Rg[:, 0:3], R_o[:, 0:3]) < TOL_ASM
    assert rel_err(Rg[:, 3], R_o[:, 3]) < TOL_ASM
    cg = corr.cpu().numpy()
    assert rel_err(cg[:, 0:3], corr_o[:, 0:3]) < TOL_ASM
    assert rel_err(cg[:, 3], corr_o[:, 3]) < TOL_ASM
    Kg = gpu_K_scipy(prob, K)
    for part, (ri, ci) in {"A": (slice(0, 3), slice(0, 3)), "B": (slice(0, 3), 3),
                           "C": (3, slice(0, 3)), "D": (3, 3)}.items():
        idx = np.arange(4 * mesh.n_nodes).reshape(-1, 4)
        rows = idx[:, ri].ravel()
        cols = idx[:, ci].ravel()
        g = Kg[rows][:, cols].toarray()
        o = K_o[rows][:, cols].toarray()
        assert rel_err(g, o) < TOL_ASM, part


def test_assembly_is_bitwise_reproducible(problems):
    prob, mesh, mat, ti, disc = problems("cube-comp")
    sn, it = states(mesh, 41)
    st = gpu_state(prob, sn, it)
    fl = V.ASM_RESIDUAL | V.ASM_TANGENT
    K1, R1, _ = prob.assemble(st, gpu_ti(ti, 0.0), fl)
    K2, R2, _ = prob.assemble(st, gpu_ti(ti, 0.0), fl)
    assert torch.equal(R1, R2)
    for a, b in ((K1.A, K2.A), (K1.B, K2.B), (K1.C, K2.C), (K1.D, K2.D)):
        assert torch.equal(a, b)


@pytest.mark.parametrize("name", ["cube-comp", "tube-hgo", "strip-hgo"])
def test_block_products_match_oracle_matrix(problems, name):
    prob, mesh, mat, ti, disc = problems(name)
    sn, it = states(mesh, 51)
    am, af, gm = E.genalpha(ti.rho_inf)
    K_o = disc.tangent(NW.stage(sn, it, am, af), (am, af, gm, ti.dt))
    K = upload_K(prob, K_o)
    n = mesh.n_nodes
    rng = np.random.default_rng(1)
    x = rng.standard_normal(4 * n)
    xf = torch.from_numpy(x).cuda()
    y = prob.spmv(K, V.OP_FULL, xf.view(n, 4)).cpu().numpy().ravel()
    assert rel_err(y, K_o @ x) < 1e-13
    xv, xp = x.reshape(n, 4)[:, :3].copy(), x.reshape(n, 4)[:, 3].copy()
    iv = np.arange(4 * n).reshape(n, 4)[:, :3].ravel()
    ip = np.arange(4 * n).reshape(n, 4)[:, 3]
    Ao, Bo, Co, Do = K_o[iv][:, iv], K_o[iv][:, ip], K_o[ip][:, iv], K_o[ip][:, ip]
    xvt = torch.from_numpy(xv).cuda()
    xpt = torch.from_numpy(xp).cuda()
    assert rel_err(prob.spmv(K, V.OP_A, xvt).cpu().numpy().ravel(), Ao @ xv.ravel()) < 1e-13
    assert rel_err(prob.spmv(K, V.OP_B, xpt).cpu().numpy().ravel(), Bo @ xp) < 1e-13
    assert rel_err(prob.spmv(K, V.OP_C, xvt).cpu().numpy().ravel(), Co @ xv.ravel()) < 1e-13
    assert rel_err(prob.spmv(K, V.OP_D, xpt).cpu().numpy().ravel(), Do @ xp) < 1e-13


def _prepared(prob, mesh, ti, disc, seed, mirror32=False, nonzero_rk=True, zero_accel=False):
    sn, it = states(mesh, seed)
    if zero_accel:   # v-dot = 0 at both levels: the inertial term rho v-dot dJ/du drops out of A
        sn["dv"][:] = 0.0
        it["dv"][:] = 0.0
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    for k in ("u", "v", "du", "dv"):
        sn[k][vm] = 0.0
        it[k][vm] = 0.0
    st = gpu_state(prob, sn, it)
    t_n = 0.0
    K, R, corr = prob.assemble(st, gpu_ti(ti, t_n), V.ASM_RESIDUAL | V.ASM_TANGENT | V.ASM_RKCORR)
    if mirror32:
        K = _with_mirrors(prob, K)
    rhs = prob.prepare(K, R, corr, 1e-15, mirror32)
    am, af, gm = E.genalpha(ti.rho_inf)
    sto = NW.stage(sn, it, am, af)
    load = NW.load_scale(ti, t_n + af * ti.dt)
    K_o, rhs_o, _, _ = NW.linear_system(disc, ti, sto, load, rk_corr=True)
    Kd, rd = AS.apply_dirichlet(K_o, rhs_o, disc.dof_dir)
    W = AS.scaling(Kd)
    Ks = Kd.multiply(W[:, None]).multiply(W[None, :]).tocsr()
    return st, K, rhs, Ks, W * rd, W, (sn, it, sto)


@pytest.mark.parametrize("name", ["cube-nu0499", "cube-incomp", "tube-hgo", "strip-hgo", "cube-fan"])
def test_schur_hat_matches_oracle(problems, name):
    """S^ = D - C diag(A)^-1 B (section 4.2) of the oracle's scaled system, formed with scipy."""
    import scipy.sparse as sp
    prob, mesh, mat, ti, disc = problems(name)
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 61)
    S, Sd, sdinv = prob.schur_hat(K)
    A, B, Cm, D, iv, ip = AS.split_blocks(Ks)
    dA = A.diagonal()
    Sh = (D - Cm @ sp.diags(np.where(dA != 0.0, 1.0 / np.where(dA != 0.0, dA, 1.0), 0.0)) @ B).tocsr()
    h = prob.host
    n = mesh.n_nodes
    W2 = prob.shat_width
    rows = np.repeat(np.arange(n), W2)
    Sg = (sp.coo_matrix((S.cpu().numpy().ravel(), (rows, h["shat_col"])), shape=(n, n))
          + sp.diags(Sd.cpu().numpy())).tocsr()
    scale = np.abs(Sh).max()
    assert np.abs(Sg - Sh).max() <= 1e-12 * scale
    dS = Sh.diagonal()
    expect = np.where((dS != 0.0) & np.isfinite(dS), 1.0 / np.where(dS != 0.0, dS, 1.0), 1.0)
    assert rel_err(sdinv.cpu().numpy(), expect) < 1e-12


@pytest.mark.parametrize("name", ["cube-nu0499", "tube-hgo", "strip-hgo", "cube-fan"])
@pytest.mark.parametrize("fp32", [False, True])
def test_shat_product_matches_oracle(problems, name, fp32):
    """y = S^ x by the product kernel of the Schur preconditioner's CG steps
    against the oracle's S^ (scipy) times the same x; FP32 storage with FP64
    accumulation to 1e-5 of the largest |S^| |x| row sum."""
    import scipy.sparse as sp
    prob, mesh, mat, ti, disc = problems(name)
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 62)
    S, Sd, _ = prob.schur_hat(K)
    A, B, Cm, D, iv, ip = AS.split_blocks(Ks)
    Sh = (D - Cm @ sp.diags(1.0 / A.diagonal()) @ B).tocsr()
    x = np.random.default_rng(3).standard_normal(mesh.n_nodes)
    xt = torch.from_numpy(x).to("cuda:0")
    if fp32:
        y = prob.shat_spmv(S.float(), Sd.float(), xt.float()).double().cpu().numpy()
        x = xt.float().double().cpu().numpy()
    else:
        y = prob.shat_spmv(S, Sd, xt).cpu().numpy()
    ref = Sh @ x
    scale = (abs(Sh) @ np.abs(x)).max()
    assert np.abs(y - ref).max() <= (1e-5 if fp32 else 1e-11) * scale


@pytest.mark.parametrize("method", [V.SHAT_CG, V.SHAT_CHEBYSHEV])
def test_compact_shat_offsets_give_identical_results(method):
    """The S^ products read 2-byte column offsets when the mesh has them and
    4-byte columns otherwise; both address the same entries in the same
    order, so products and solves agree bit for bit."""
    mesh, mat, ti = case("cube-nu0499")
    pa = V.Problem(mesh, mat, "cuda:0")
    pb = V.Problem(mesh, mat, "cuda:0", compact_shat=False)
    assert pa.d["shat_off"] is not None and pb.d["shat_off"] is None
    sn, it = states(mesh, 63)
    out = []
    for prob in (pa, pb):
        st = gpu_state(prob, sn, it)
        K, R, corr = prob.assemble(st, gpu_ti(ti, 0.0), V.ASM_RESIDUAL | V.ASM_TANGENT | V.ASM_RKCORR)
        rhs = prob.prepare(K, R, corr)
        S, Sd, _ = prob.schur_hat(K)
        xs = torch.linspace(-1.0, 1.0, mesh.n_nodes, dtype=torch.float64, device="cuda:0")
        y = prob.shat_spmv(S, Sd, xs)
        x, stats = prob.solve_scaled(K, rhs, V.solver_opts(rtol=1e-8, shat_method=method, shat_degree=8))
        out.append((y, x, stats["it_S"]))
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1]) and out[0][2] == out[1][2]


def _with_mirrors(prob, K):
    K2 = prob.new_matrix(mirror32=True)
    for a, b in ((K2.A, K.A), (K2.B, K.B), (K2.C, K.C), (K2.D, K.D)):
        a.copy_(b)
    return K2


@pytest.mark.parametrize("name", ["cube-comp", "tube-hgo", "strip-hgo"])
def test_dirichlet_and_scaling_match_oracle(problems, name):
    prob, mesh, mat, ti, disc = problems(name)
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 61, mirror32=True)
    torch.cuda.synchronize()
    assert rel_err(K.W.cpu().numpy().ravel(), W) < 1e-13
    assert rel_err(rhs.cpu().numpy().ravel(), rs) < TOL_ASM
    Kg = gpu_K_scipy(prob, K)
    assert rel_err(Kg.toarray() if Kg.shape[0] < 3000 else Kg.data, Ks.toarray() if Kg.shape[0] < 3000 else Ks.data) < TOL_ASM
    for a32, a64 in ((K.A32, K.A), (K.B32, K.B), (K.C32, K.C), (K.D32, K.D)):
        assert torch.equal(a32, a64.float())


@pytest.mark.parametrize("precond,max_outer", [(V.PC_LDU, 1), (V.PC_UPPER, 2), (V.PC_LOWER, 2)])
@pytest.mark.parametrize("orth,shat,method", [(V.ORTH_CGS2, 0, V.SHAT_CHEBYSHEV), (V.ORTH_MGS, 0, V.SHAT_CHEBYSHEV),
                                              (V.ORTH_CGS2, 6, V.SHAT_CHEBYSHEV), (V.ORTH_CGS1, 0, V.SHAT_CHEBYSHEV),
                                              (V.ORTH_CGS_IFNEEDED, 0, V.SHAT_CHEBYSHEV),
                                              (V.ORTH_CGS_IFNEEDED, 6, V.SHAT_CHEBYSHEV),
                                              (V.ORTH_CGS1, 16, V.SHAT_CG)])
def test_nested_solve_matches_lu(problems, precond, max_outer, orth, shat, method):
    import scipy.sparse.linalg as spla
    prob, mesh, mat, ti, disc = problems("cube-comp")
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 71)
    opts = V.solver_opts(rtol=1e-9, rtol_A=1e-13, rtol_S=1e-13, rtol_I=1e-14, maxit=50, maxit_A=400,
                         maxit_S=400, maxit_I=400, precond=precond, orth=orth, shat_degree=shat,
                         shat_method=method)
    x, stats = prob.solve_scaled(K, rhs, opts)
    xg = x.cpu().numpy().ravel()
    xo = spla.splu(Ks.tocsc()).solve(rs)
    print(f"[solve] precond={precond} orth={orth} stats={stats}", flush=True)
    assert stats["n_outer"] <= max_outer
    assert np.linalg.norm(Ks @ xg - rs) <= 1e-9 * np.linalg.norm(rs)
    assert np.linalg.norm(xg - xo) <= 1e-7 * np.linalg.norm(xo)


@pytest.mark.parametrize("name,precision", [("cube-comp", V.FP64), ("tube-hgo", V.FP64), ("strip-hgo", V.FP64),
                                            ("cube-nu0499", V.MIXED), ("strip-hgo", V.MIXED)])
def test_solve_unscaled_matches_oracle(problems, name, precision):
    """solve(K, R) -> Delta (vms_solve, section 3.3 step 5 with section 4.1's
    scaling): K and R as assembled go in, Delta = W x* comes out; compared with
    the oracle's scaled sparse LU (oracle.newton.solve_scaled) to a relative
    residual of 1e-8 in the scaled system and 1e-7 in Delta.  K is left
    holding W K W, and the phase times nest as documented."""
    prob, mesh, mat, ti, disc = problems(name)
    mixed = precision == V.MIXED
    sn, it = states(mesh, 101)
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    for k in ("u", "v", "du", "dv"):
        sn[k][vm] = 0.0
        it[k][vm] = 0.0
    st = gpu_state(prob, sn, it)
    K, R, corr = prob.assemble(st, gpu_ti(ti, 0.0), V.ASM_RESIDUAL | V.ASM_TANGENT | V.ASM_RKCORR)
    if mixed:
        K = _with_mirrors(prob, K)
    opts = (V.solver_opts(rtol=1e-10, rtol_A=1e-5, rtol_S=1e-5, rtol_I=1e-4, precision=V.MIXED, a_krylov=V.AK_CG,
                          cg_symmetrise=0, maxit=400)
            if mixed else V.solver_opts(rtol=1e-10, rtol_A=1e-12, rtol_S=1e-12, rtol_I=1e-13))
    delta, stats = prob.solve(K, R, opts, corr=corr)
    am, af, gm = E.genalpha(ti.rho_inf)
    sto = NW.stage(sn, it, am, af)
    K_o, rhs_o, _, _ = NW.linear_system(disc, ti, sto, NW.load_scale(ti, af * ti.dt), rk_corr=True)
    d_o = NW.solve_scaled(K_o, rhs_o, disc.dof_dir)
    Kd, rd = AS.apply_dirichlet(K_o, rhs_o, disc.dof_dir)
    W = AS.scaling(Kd)
    Ks = Kd.multiply(W[:, None]).multiply(W[None, :]).tocsr()
    dg = delta.cpu().numpy().ravel()
    xs = dg / W
    print(f"[solve] {name} precision={precision} {stats}", flush=True)
    assert stats["status"] == 0 and stats["phases_timed"] == 1
    assert np.all(dg[disc.dof_dir] == 0.0)
    assert np.linalg.norm(Ks @ xs - W * rd) <= 1e-8 * np.linalg.norm(W * rd)
    assert np.linalg.norm(dg - d_o) <= 1e-7 * np.linalg.norm(d_o)
    # K now holds W K W, and K.W the scaling
    assert rel_err(K.W.cpu().numpy().ravel(), W) < 1e-13
    Kg = gpu_K_scipy(prob, K)
    assert abs(Kg - Ks).max() <= TOL_ASM * abs(Ks).max()
    # phases: scaling, set-up and the outer solve are timed; A, Schur and inner solves nest in it
    for k in ("ms_scale", "ms_setup", "ms_outer", "ms_A", "ms_S", "ms_inner"):
        assert stats[k] > 0.0, k
    assert stats["ms_outer"] >= stats["ms_A"] + stats["ms_S"] - 1e-3
    assert stats["ms_S"] >= stats["ms_inner"] - 1e-3


@pytest.mark.parametrize("precision", [V.FP64, V.MIXED])
@pytest.mark.parametrize("shat,method", [(0, V.SHAT_CHEBYSHEV), (16, V.SHAT_CG)])
def test_block_diagonal_solve_matches_lu(problems, precision, shat, method):
    """The block-diagonal partial factorization (section 4.4 remark on D):
    with D != 0 it has no small iteration bound, so the outer count is held to
    that of the oracle's FGMRES with the exact block-diagonal preconditioner
    on the same scaled system (plus two for the inexact inner solves), and the
    solution must be the LU one."""
    import scipy.sparse.linalg as spla
    from oracle import krylov as KR
    prob, mesh, mat, ti, disc = problems("cube-comp")
    mixed = precision == V.MIXED
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 71, mirror32=mixed)
    A, B, Cb, Db, iv, ip = AS.split_blocks(Ks)
    perm = np.concatenate([iv, ip])
    Kp = Ks[perm][:, perm].tocsr()
    P = KR.block_preconditioner(A, B, Cb, Db, "diag")
    _, its_oracle, _ = KR.fgmres(lambda z: Kp @ z, rs[perm], P, rtol=1e-9, maxit=400)
    inner = dict(rtol_A=1e-6, rtol_S=1e-6, rtol_I=1e-6) if mixed else dict(rtol_A=1e-13, rtol_S=1e-13,
                                                                            rtol_I=1e-14)
    opts = V.solver_opts(rtol=1e-9, maxit=400, maxit_A=400, maxit_S=400, maxit_I=400, precond=V.PC_DIAG,
                         precision=precision, shat_degree=shat, shat_method=method, **inner)
    x, stats = prob.solve_scaled(K, rhs, opts)
    xg = x.cpu().numpy().ravel()
    xo = spla.splu(Ks.tocsc()).solve(rs)
    print(f"[diag] precision={precision} oracle its={its_oracle} stats={stats}", flush=True)
    assert stats["status"] == 0
    # FP64 inner solves at 1e-13 act as exact ones; the FP32 levels at 1e-6 may cost a few more
    assert stats["n_outer"] <= (2 * its_oracle + 2 if mixed else its_oracle + 2)
    assert np.linalg.norm(Ks @ xg - rs) <= 1e-9 * np.linalg.norm(rs)
    assert np.linalg.norm(xg - xo) <= 1e-7 * np.linalg.norm(xo)


def test_predictor_literal_factors(problems):
    """Predictor stage of section 3.3 at rho_inf = 0.5: y_(0) = y_n and
    y-dot_(0) = (gamma - 1)/gamma y-dot_n = -y-dot_n / 2 (gamma = 2/3), with
    the literal factor; prescribed components take u = g(t_{n+1}), v = u-dot =
    g-dot, v-dot = 0."""
    prob, mesh, mat, ti, disc = problems("tube-hgo")
    sn, it = states(mesh, 17)
    st = gpu_state(prob, sn, it)
    t_n = 0.3
    prob.predictor(st, gpu_ti(ti, t_n))
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    assert vm.any() and (~vm).any()
    for k in ("u", "p", "v"):
        want = sn[k].copy()
        if k in ("u", "v"):
            want[vm] = (mesh.dir_vel * (t_n + ti.dt) if k == "u" else mesh.dir_vel)[vm]
        assert np.array_equal(st[k].cpu().numpy(), want), k
    for k in ("du", "dp", "dv"):
        want = -0.5 * sn[k]
        if k == "du":
            want[vm] = mesh.dir_vel[vm]
        if k == "dv":
            want[vm] = 0.0
        assert np.abs(st[k].cpu().numpy() - want).max() <= 1e-15 * np.abs(sn[k]).max(), k


@pytest.mark.parametrize("name", ["cube-nu0499", "cube-incomp", "tube-hgo", "strip-hgo", "cube-fan"])
@pytest.mark.parametrize("precision", [V.FP64, V.MIXED])
@pytest.mark.parametrize("shat,shat_method", [(0, V.SHAT_CHEBYSHEV), (6, V.SHAT_CHEBYSHEV), (6, V.SHAT_CG)])
def test_solve_reaches_requested_residual(problems, name, precision, shat, shat_method):
    import scipy.sparse.linalg as spla
    prob, mesh, mat, ti, disc = problems(name)
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 81, mirror32=(precision == V.MIXED))
    if precision == V.MIXED:
        opts = V.solver_opts(rtol=1e-8, rtol_A=1e-5, rtol_S=1e-5, rtol_I=1e-3, precision=V.MIXED,
                             shat_degree=shat, shat_method=shat_method)
    else:
        opts = V.solver_opts(rtol=1e-8, shat_degree=shat, shat_method=shat_method)
    x, stats = prob.solve_scaled(K, rhs, opts)
    xg = x.cpu().numpy().ravel()
    print(f"[solve] {name} precision={precision} stats={stats}", flush=True)
    res = np.linalg.norm(Ks @ xg - rs) / np.linalg.norm(rs)
    assert res <= 2e-8
    xo = spla.splu(Ks.tocsc()).solve(rs)
    assert np.linalg.norm(xg - xo) <= 1e-5 * np.linalg.norm(xo)


@pytest.mark.parametrize("name", ["cube-nu0499", "tube-hgo", "strip-hgo", "cube-fan"])
@pytest.mark.parametrize("precision", [V.FP64, V.MIXED])
@pytest.mark.parametrize("a_krylov,sym", [(V.AK_CG_INNER, 1), (V.AK_CG, 1), (V.AK_CG, 0)])
def test_cg_levels_solve_matches_lu(problems, name, precision, a_krylov, sym):
    """CG on (A + A^T)/2 at the A-levels (the inner-solver choice suggested in
    the paper's conclusions) only changes the preconditioner: the outer FGMRES
    still reaches the requested residual of the unsymmetrised system."""
    import scipy.sparse.linalg as spla
    prob, mesh, mat, ti, disc = problems(name)
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 83, mirror32=(precision == V.MIXED))
    opts = V.solver_opts(rtol=1e-8, precision=precision, shat_degree=6, a_krylov=a_krylov, cg_symmetrise=sym)
    x, stats = prob.solve_scaled(K, rhs, opts)
    xg = x.cpu().numpy().ravel()
    print(f"[solve] {name} precision={precision} a_krylov={a_krylov} sym={sym} stats={stats}", flush=True)
    assert np.linalg.norm(Ks @ xg - rs) <= 2e-8 * np.linalg.norm(rs)
    xo = spla.splu(Ks.tocsc()).solve(rs)
    assert np.linalg.norm(xg - xo) <= 1e-5 * np.linalg.norm(xo)
    assert stats["n_I_solves"] > 0 and stats["it_I"] > 0


@pytest.mark.parametrize("name", ["cube-nu0499", "strip-hgo"])
@pytest.mark.parametrize("precision,a_krylov", [(V.FP64, V.AK_GMRES), (V.MIXED, V.AK_CG)])
def test_relaxed_inner_tolerance_solve_matches_lu(problems, name, precision, a_krylov):
    """With the inner tolerance relaxed as the Schur level converges, the
    nested preconditioner changes but the outer FGMRES still reaches the
    requested residual of the oracle's system and its LU solution."""
    import scipy.sparse.linalg as spla
    prob, mesh, mat, ti, disc = problems(name)
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 85, mirror32=(precision == V.MIXED))
    res = {}
    for relax in (0, 1):   # relaxation off (the paper's fixed inner tolerance) and on
        opts = V.solver_opts(rtol=1e-8, rtol_I=1e-4, precision=precision, a_krylov=a_krylov, cg_symmetrise=0,
                             relax_inner=relax)
        x, stats = prob.solve_scaled(K, rhs, opts)
        xg = x.cpu().numpy().ravel()
        print(f"[relax] {name} precision={precision} relax={relax} stats={stats}", flush=True)
        assert np.linalg.norm(Ks @ xg - rs) <= 2e-8 * np.linalg.norm(rs)
        xo = spla.splu(Ks.tocsc()).solve(rs)
        assert np.linalg.norm(xg - xo) <= 1e-5 * np.linalg.norm(xo)
        res[relax] = stats
    assert res[0]["status"] == 0 and res[1]["status"] == 0


@pytest.mark.parametrize("name", ["cube-nu0499", "tube-hgo", "strip-hgo"])
@pytest.mark.parametrize("precision,a_krylov", [(V.FP64, V.AK_GMRES), (V.MIXED, V.AK_CG)])
@pytest.mark.parametrize("shat_method,shat_degree", [(V.SHAT_CG, 6), (V.SHAT_NONE, 0), (V.SHAT_CG, 0)])
def test_pressure_mass_schur_preconditioner_solve_matches_lu(problems, name, precision, a_krylov, shat_method,
                                                             shat_degree):
    """The pressure-mass term of the Schur preconditioner (added to CG steps on
    S^ or to diag(S^)^-1, or alone) changes only the preconditioner: the solve
    reaches the requested residual and the oracle's LU solution."""
    import scipy.sparse.linalg as spla
    prob, mesh, mat, ti, disc = problems(name)
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 86, mirror32=(precision == V.MIXED))
    opts = V.solver_opts(rtol=1e-8, precision=precision, a_krylov=a_krylov, cg_symmetrise=0,
                         shat_method=shat_method, shat_degree=shat_degree, schur_mass=1.0)
    x, stats = prob.solve_scaled(K, rhs, opts)
    xg = x.cpu().numpy().ravel()
    print(f"[mass] {name} precision={precision} method={shat_method} degree={shat_degree} stats={stats}", flush=True)
    assert stats["status"] == 0
    assert np.linalg.norm(Ks @ xg - rs) <= 2e-8 * np.linalg.norm(rs)
    xo = spla.splu(Ks.tocsc()).solve(rs)
    assert np.linalg.norm(xg - xo) <= 1e-5 * np.linalg.norm(xo)


@pytest.mark.parametrize("precision", [V.FP64, V.MIXED])
def test_cg_product_launch_timing(problems, precision):
    """With launch timing on, every CG product launch that does the product is
    timed and counted: one per CG iteration of the two A-levels, none for the
    launches that only find the level converged."""
    prob, mesh, mat, ti, disc = problems("cube-nu0499")
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 84, mirror32=(precision == V.MIXED))
    opts = V.solver_opts(rtol=1e-8, precision=precision, a_krylov=V.AK_CG, cg_symmetrise=0)
    prob.set_timing(True)
    x, stats = prob.solve_scaled(K, rhs, opts)
    ms, cnt = prob.kernel_time(fp32=precision == V.MIXED)
    other = prob.kernel_time(fp32=precision != V.MIXED)
    prob.set_timing(False)
    print(f"[timing] precision={precision} launches={cnt} ms={ms:.3f} stats={stats}", flush=True)
    assert cnt == stats["it_A"] + stats["it_I"] > 0
    assert ms > 0.0 and other == (0.0, 0)


@pytest.mark.parametrize("a_krylov,sym", [(V.AK_CG_INNER, 1), (V.AK_CG, 1), (V.AK_CG, 0)])
def test_cg_exact_on_symmetric_A(problems, a_krylov, sym):
    """With zero accelerations A is symmetric, so (A + A^T)/2 = A: CG solved
    to 1e-14 makes the full block factorization exact (Algorithm 1), and the
    outer FGMRES stops after one iteration, as it does with GMRES."""
    import scipy.sparse.linalg as spla
    prob, mesh, mat, ti, disc = problems("cube-comp")
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 71, zero_accel=True)
    A = AS.split_blocks(Ks)[0]
    assert abs(A - A.T).max() <= 1e-14 * abs(A).max()
    opts = V.solver_opts(rtol=1e-9, rtol_A=1e-13, rtol_S=1e-13, rtol_I=1e-14, maxit=50, maxit_A=400,
                         maxit_S=400, maxit_I=400, shat_degree=6, a_krylov=a_krylov, cg_symmetrise=sym)
    x, stats = prob.solve_scaled(K, rhs, opts)
    xg = x.cpu().numpy().ravel()
    print(f"[solve] symmetric A, a_krylov={a_krylov} sym={sym} stats={stats}", flush=True)
    assert stats["n_outer"] == 1
    xo = spla.splu(Ks.tocsc()).solve(rs)
    assert np.linalg.norm(xg - xo) <= 1e-7 * np.linalg.norm(xo)


def test_shat_cg_steps_approach_exact_shat(problems):
    """k CG steps on S^ converge to S^-1 as k grows: with k = 60 and exact
    inner and A-solves, the one Schur solve of the nested solve takes as many
    iterations (within one) as the oracle's S-GMRES on the same right-hand
    side (Algorithm 1, steps 1-2 applied to the first outer Krylov vector)
    preconditioned by an exact S^ solve.  Steepest descent or a wrong CG
    coefficient would need several more."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from oracle import krylov as KR
    prob, mesh, mat, ti, disc = problems("cube-nu0499")
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 85)
    opts = V.solver_opts(rtol=1e-9, rtol_A=1e-13, rtol_S=1e-10, rtol_I=1e-13, maxit_S=400, maxit_A=400,
                         maxit_I=400, shat_degree=60, shat_method=V.SHAT_CG)
    x, stats = prob.solve_scaled(K, rhs, opts)
    print(f"[solve] S^ CG(60) stats={stats}", flush=True)
    assert stats["n_outer"] == 1 and stats["n_S_solves"] == 1
    A, B, Cm, D, iv, ip = AS.split_blocks(Ks)
    Sh = (D - Cm @ sp.diags(1.0 / A.diagonal()) @ B).tocsc()
    luA, luS = spla.splu(A.tocsc()), spla.splu(Sh)
    v0 = rs / np.linalg.norm(rs)
    bS = v0[ip] - Cm @ luA.solve(v0[iv])
    its = KR.fgmres(lambda v: D @ v - Cm @ luA.solve(B @ v), bS, precond=luS.solve, rtol=1e-10, maxit=400)[1]
    print(f"[solve] oracle S-GMRES with exact S^: {its} iterations", flush=True)
    assert abs(stats["it_S"] - its) <= 1
    xo = spla.splu(Ks.tocsc()).solve(rs)
    assert np.linalg.norm(x.cpu().numpy().ravel() - xo) <= 1e-7 * np.linalg.norm(xo)


@pytest.mark.parametrize("name", ["cube-comp", "cube-nu0499"])
def test_simple_matches_oracle_iterations(problems, name):
    """SIMPLE (section 4.3) with its A- and S^-solves run to 1e-13 takes as
    many outer FGMRES iterations (within one) as the oracle's FGMRES with the
    exact SIMPLE factors, and reaches the LU solution."""
    import scipy.sparse.linalg as spla
    from oracle import krylov as KR
    prob, mesh, mat, ti, disc = problems(name)
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 87)
    opts = V.solver_opts(rtol=1e-9, rtol_A=1e-13, rtol_S=1e-13, maxit=100, maxit_A=400, maxit_S=400,
                         precond=V.PC_SIMPLE)
    x, stats = prob.solve_scaled(K, rhs, opts)
    print(f"[solve] SIMPLE {name} stats={stats}", flush=True)
    A, B, Cm, D, iv, ip = AS.split_blocks(Ks)
    perm = np.concatenate([iv, ip])
    Kp = Ks[perm][:, perm].tocsr()
    _, its, _ = KR.fgmres(lambda z: Kp @ z, rs[perm], KR.simple_preconditioner(A, B, Cm, D), rtol=1e-9, maxit=100)
    print(f"[solve] oracle SIMPLE: {its} outer iterations", flush=True)
    assert abs(stats["n_outer"] - its) <= 1
    assert stats["n_I_solves"] == 0 and stats["n_S_solves"] == stats["n_outer"]
    xo = spla.splu(Ks.tocsc()).solve(rs)
    assert np.linalg.norm(x.cpu().numpy().ravel() - xo) <= 1e-7 * np.linalg.norm(xo)


@pytest.mark.parametrize("precond", [V.PC_LDU, V.PC_SIMPLE])
@pytest.mark.parametrize("precision", [V.FP64, V.MIXED])
def test_single_shat_schur_step_reaches_lu(problems, precond, precision):
    """The Schur step as one application of the S^ preconditioner (no inner
    solve, the loosest end of section 4.4) is still a valid preconditioner:
    the outer FGMRES reaches the requested residual and the LU solution."""
    import scipy.sparse.linalg as spla
    prob, mesh, mat, ti, disc = problems("cube-nu0499")
    st, K, rhs, Ks, rs, W, _ = _prepared(prob, mesh, ti, disc, 89, mirror32=(precision == V.MIXED))
    opts = V.solver_opts(rtol=1e-8, precond=precond, precision=precision, schur_solve=V.SCHUR_SHAT)
    x, stats = prob.solve_scaled(K, rhs, opts)
    print(f"[solve] S^-only precond={precond} precision={precision} stats={stats}", flush=True)
    assert stats["n_I_solves"] == 0 and stats["it_S"] == 0 and stats["n_S_solves"] == stats["n_outer"]
    xg = x.cpu().numpy().ravel()
    assert np.linalg.norm(Ks @ xg - rs) <= 2e-8 * np.linalg.norm(rs)
    xo = spla.splu(Ks.tocsc()).solve(rs)
    assert np.linalg.norm(xg - xo) <= 1e-5 * np.linalg.norm(xo)


def test_newton_update_matches_oracle(problems):
    prob, mesh, mat, ti, disc = problems("cube-comp")
    sn, it = states(mesh, 91)
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    for k in ("u", "v", "du", "dv"):
        sn[k][vm] = 0.0
        it[k][vm] = 0.0
    st = gpu_state(prob, sn, it)
    rng = np.random.default_rng(5)
    n = mesh.n_nodes
    x = rng.standard_normal((n, 4))
    x[mesh.dir_mask.astype(bool)] = 0.0
    W = rng.uniform(0.5, 2.0, (n, 4))
    K = prob.new_matrix()
    K.W.copy_(torch.from_numpy(W))
    prob.newton_update(st, gpu_ti(ti, 0.0), K, torch.from_numpy(x / W).cuda())
    am, af, gm = E.genalpha(ti.rho_inf)
    sto = NW.stage(sn, it, am, af)
    out, _ = NW.newton_update(disc, ti, it, x.ravel(), sto["du"] - sto["v"])
    for k in ("u", "p", "v", "du", "dp", "dv"):
        assert rel_err(st[k].cpu().numpy(), out[k]) < 1e-13, k


def _run_steps(prob, mesh, ti, n_steps, nopts, sopts, allow_nc=False):
    st = prob.new_state()
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    for key in ("v_n", "du_n"):
        a = st[key].cpu().numpy()
        a[vm] = mesh.dir_vel[vm]
        st[key].copy_(torch.from_numpy(a))
    hist = []
    K = None
    for s in range(n_steps):
        stats, K = prob.step(st, V.time_int(ti.dt, ti.rho_inf, s * ti.dt, ti.n_steps * ti.dt), nopts, sopts, K,
                             allow_nc=allow_nc)
        hist.append(stats)
        if stats["status"] != 0:
            print(f"[step {s}] status {stats['status']} res={stats['res_norm']}", flush=True)
            break
        prob.roll(st)
    return st, hist


@pytest.mark.parametrize("N,nu,n_steps,variant", [(4, None, 1, "gmres"), (4, 0.45, 3, "gmres"), (3, 0.5, 2, "gmres"),
                                                   (4, 0.45, 3, "cg"), (4, 0.45, 3, "simple")])
def test_time_steps_match_oracle(N, nu, n_steps, variant):
    """Whole time steps against the oracle's: GMRES A-levels; CG A-levels
    (on A itself); and the SIMPLE preconditioner."""
    mesh, mat, ti = synth.cube_case(N, nu=nu, n_steps=n_steps)
    prob = V.Problem(mesh, mat, "cuda:0")
    nopts = V.newton_opts(tol_R=1e-10, l_max=10)
    extra = {"gmres": {}, "cg": dict(a_krylov=V.AK_CG, cg_symmetrise=0), "simple": dict(precond=V.PC_SIMPLE)}[variant]
    sopts = V.solver_opts(rtol=1e-10, rtol_A=1e-10, rtol_S=1e-10, rtol_I=1e-12, **extra)
    st, hist = _run_steps(prob, mesh, ti, n_steps, nopts, sopts)
    disc = AS.Discretization(mesh, mat)
    so = NW.rest_state(mesh)
    for s in range(n_steps):
        so, info = NW.time_step(disc, ti, so, s * ti.dt, tol_R=1e-10)
        print(f"[step {s}] gpu newton={hist[s]['n_newton']} res={hist[s]['res_norm']} oracle={info['norms']}",
              flush=True)
        assert hist[s]["n_newton"] == info["n_newton"]
    for k in ("u", "p", "v", "du", "dp", "dv"):
        assert rel_err(st[k].cpu().numpy(), so[k]) < 1e-7, k


@pytest.mark.parametrize("a_krylov", [V.AK_GMRES, V.AK_CG])
def test_mixed_precision_time_step_error(a_krylov):
    """The mixed form (FP32 intermediate and inner levels; GMRES or, as the
    bench runs it, CG on A itself) reaches the oracle's FP64 time steps."""
    mesh, mat, ti = synth.cube_case(4, nu=0.499, n_steps=2)
    prob = V.Problem(mesh, mat, "cuda:0")
    nopts = V.newton_opts(tol_R=1e-8, l_max=10)
    sopts = V.solver_opts(rtol=1e-8, rtol_A=1e-5, rtol_S=1e-5, rtol_I=1e-3, precision=V.MIXED, a_krylov=a_krylov,
                          cg_symmetrise=0)
    st, hist = _run_steps(prob, mesh, ti, 2, nopts, sopts)
    disc = AS.Discretization(mesh, mat)
    so = NW.rest_state(mesh)
    for s in range(2):
        so, info = NW.time_step(disc, ti, so, s * ti.dt, tol_R=1e-8)
    err = rel_err(st["u"].cpu().numpy(), so["u"])
    print(f"[mixed] displacement error vs FP64 oracle = {err:.3e}; stats={hist[-1]}", flush=True)
    assert all(h["status"] == 0 for h in hist)
    assert err < 1e-6


@pytest.mark.parametrize("precision,a_krylov", [(V.FP64, V.AK_GMRES), (V.MIXED, V.AK_CG)])
def test_strip_time_steps_match_oracle(precision, a_krylov):
    """Three time steps of the small eighth-strip (incompressible HGO with
    dispersion, symmetry conditions, traction on the loading face) against the
    oracle's: FP64 with GMRES A-levels, and the mixed form with CG on A as the
    bench runs it."""
    mesh, mat, ti = STRIP()
    prob = V.Problem(mesh, mat, "cuda:0")
    mixed = precision == V.MIXED
    nopts = V.newton_opts(tol_R=1e-8 if mixed else 1e-10, l_max=10)
    if mixed:
        sopts = V.solver_opts(rtol=1e-8, rtol_A=1e-5, rtol_S=1e-5, rtol_I=1e-3, precision=V.MIXED,
                              a_krylov=a_krylov, cg_symmetrise=0)
    else:
        sopts = V.solver_opts(rtol=1e-10, rtol_A=1e-10, rtol_S=1e-10, rtol_I=1e-12)
    st, hist = _run_steps(prob, mesh, ti, 3, nopts, sopts)
    disc = AS.Discretization(mesh, mat)
    so = NW.rest_state(mesh)
    for s in range(3):
        so, info = NW.time_step(disc, ti, so, s * ti.dt, tol_R=nopts.tol_R)
        print(f"[strip step {s}] gpu newton={hist[s]['n_newton']} res={hist[s]['res_norm']} "
              f"oracle={info['norms']}", flush=True)
        assert hist[s]["status"] == 0
        if not mixed:
            assert hist[s]["n_newton"] == info["n_newton"]
    tol = 1e-6 if mixed else 1e-7
    for k in ("u", "p", "v") if mixed else ("u", "p", "v", "du", "dp", "dv"):
        assert rel_err(st[k].cpu().numpy(), so[k]) < tol, k


def test_lifted_predictor_and_update_match_oracle(problems):
    """Lifted Dirichlet form (reading: the prescribed motion arrives through
    R-bar_k): the predictor keeps u, v of the Dirichlet components at y_n with
    v-dot = 0, and the update moves their u by Delta u-dot = -R-bar_k/alpha_m,
    against the oracle's predictor and newton_update with lift=True."""
    prob, mesh, mat, ti, disc = problems("tube-hgo")
    sn, _ = states(mesh, 23)
    vm = mesh.dir_mask[:, 0:3].astype(bool)
    st = gpu_state(prob, sn, sn)
    t_n = 0.3
    prob.predictor(st, gpu_ti(ti, t_n), dir_lift=1)
    am, af, gm = E.genalpha(ti.rho_inf)
    ito = NW.predictor(mesh, sn, gm, t_n + ti.dt, lift=True)
    for k in ("u", "p", "v", "du", "dp", "dv"):
        assert np.abs(st[k].cpu().numpy() - ito[k]).max() <= 1e-15 * max(np.abs(ito[k]).max(), 1.0), k
    assert np.array_equal(st["u"].cpu().numpy()[vm], sn["u"][vm])
    rng = np.random.default_rng(6)
    n = mesh.n_nodes
    x = rng.standard_normal((n, 4))
    x[mesh.dir_mask.astype(bool)] = 0.0
    prob.newton_update(st, gpu_ti(ti, t_n), None, torch.from_numpy(x).cuda(), dir_lift=1)
    sto = NW.stage(sn, ito, am, af)
    out, _ = NW.newton_update(disc, ti, ito, x.ravel(), sto["du"] - sto["v"], lift=True)
    for k in ("u", "p", "v", "du", "dp", "dv"):
        assert rel_err(st[k].cpu().numpy(), out[k]) < 1e-13, k
    moved = np.abs(out["u"][vm] - sn["u"][vm]).max()
    assert moved > 0.0


@pytest.mark.parametrize("precision", [V.FP64, V.MIXED])
def test_lifted_tube_time_steps_match_oracle(precision):
    """Three time steps of a small HGO tube at the stretch rate and step of the
    full workload (stretch 1.5 over 20 steps of 0.05) with the lifted
    Dirichlet predictor, against the oracle's lifted steps."""
    mesh, mat, ti = synth.tube_case(1, 16, 20, dt=0.05, n_steps=20)
    prob = V.Problem(mesh, mat, "cuda:0")
    fib, dfib = synth.fibre_field(mesh, mesh.meta["fibre_rad"])
    prob.set_fibres(fib, dfib)
    mixed = precision == V.MIXED
    nopts = V.newton_opts(tol_R=1e-8 if mixed else 1e-10, l_max=15, dir_lift=1)
    if mixed:
        sopts = V.solver_opts(rtol=1e-8, precision=V.MIXED, a_krylov=V.AK_CG, cg_symmetrise=0)
    else:
        sopts = V.solver_opts(rtol=1e-10, rtol_A=1e-10, rtol_S=1e-10, rtol_I=1e-12)
    st, hist = _run_steps(prob, mesh, ti, 3, nopts, sopts, allow_nc=True)
    assert all(h["status"] == 0 for h in hist) and len(hist) == 3
    disc = AS.Discretization(mesh, mat)
    so = NW.rest_state(mesh)
    for s in range(3):
        so, info = NW.time_step(disc, ti, so, s * ti.dt, tol_R=nopts.tol_R, l_max=15, lift=True)
        print(f"[lifted tube step {s}] gpu newton={hist[s]['n_newton']} oracle={info['n_newton']} "
              f"gpu res={hist[s]['res_norm'][:hist[s]['n_newton'] + 1]}", flush=True)
        assert hist[s]["status"] == 0 and info["converged"]
        if not mixed:
            assert hist[s]["n_newton"] == info["n_newton"]
    tol = 1e-6 if mixed else 1e-7
    for k in ("u", "p", "v") if mixed else ("u", "p", "v", "du", "dp", "dv"):
        assert rel_err(st[k].cpu().numpy(), so[k]) < tol, k


def fan_mesh(offset=(0.0, 0.0, 0.0)):
    """A node of valence 18: the centre of a ball whose surface is the octahedron with each face
    split in four (18 surface nodes, 32 tets).  Its block row has 19 blocks, so the pattern takes
    32 slots per row and the tangent goes through the element matrices and the block gather."""
    V6 = [np.eye(3)[i] * s for i in range(3) for s in (1.0, -1.0)]
    faces = [(a, b, c) for a in (0, 1) for b in (2, 3) for c in (4, 5)]
    pts = [np.zeros(3)] + [v for v in V6]          # centre 0, octahedron vertices 1..6
    mid = {}

    def midpoint(i, j):
        key = (min(i, j), max(i, j))
        if key not in mid:
            p = pts[i] + pts[j]
            pts.append(p / np.linalg.norm(p))
            mid[key] = len(pts) - 1
        return mid[key]
    tris = []
    for a, b, c in faces:
        a, b, c = a + 1, b + 1, c + 1
        ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
        tris += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
    X = np.array(pts) + np.asarray(offset)
    tets = []
    for a, b, c in tris:
        t = [0, a, b, c]
        if np.linalg.det(np.array([X[a] - X[0], X[b] - X[0], X[c] - X[0]])) < 0.0:
            t = [0, b, a, c]
        tets.append(t)
    return X, np.array(tets, np.int32)


def _asm_case_with_fan(with_cube):
    mesh, mat, ti = synth.cube_case(3, nu=0.45, n_steps=2)
    if not with_cube:
        X, tets = fan_mesh()
        n = X.shape[0]
        m = synth.mesh.Mesh("fan", X, tets, np.zeros((0, 3), np.int32), np.zeros((0, 3)),
                            np.zeros((n, 4), np.uint8), np.zeros((n, 3)))
        return m, mat, ti
    Xf, tf = fan_mesh(offset=(10.0, 0.0, 0.0))
    n0, nf = mesh.n_nodes, Xf.shape[0]
    m = synth.mesh.Mesh("cube+fan", np.vstack([mesh.X, Xf]), np.vstack([mesh.tets, tf + n0]).astype(np.int32),
                        mesh.bfaces, mesh.traction, np.vstack([mesh.dir_mask, np.zeros((nf, 4), np.uint8)]),
                        np.vstack([mesh.dir_vel, np.zeros((nf, 3))]))
    return m, mat, ti


def test_wide_rows_assemble_through_the_element_buffer():
    """A mesh whose longest block row needs 32 slots: the tangent, residual and R-bar_k term come
    from the element kernel and the gathers, and match the oracle."""
    mesh, mat, ti = _asm_case_with_fan(False)
    prob = V.Problem(mesh, mat, "cuda:0")
    assert prob.slot_width == 32
    print(f"[assembly] fan n={mesh.n_nodes} m={mesh.n_tets} W={prob.slot_width}", flush=True)
    sn = synth.random_state(mesh.n_nodes, 61, {"u": 1e-3})
    it = synth.random_state(mesh.n_nodes, 62, {"u": 1e-3})
    st = gpu_state(prob, sn, it)
    t_n = 0.4 * ti.dt
    K, R, corr = prob.assemble(st, gpu_ti(ti, t_n), V.ASM_RESIDUAL | V.ASM_TANGENT | V.ASM_RKCORR)
    disc = AS.Discretization(mesh, mat)
    am, af, gm = E.genalpha(ti.rho_inf)
    sto = NW.stage(sn, it, am, af)
    R_o = disc.residual(sto, NW.load_scale(ti, t_n + af * ti.dt))
    K_o = disc.tangent(sto, (am, af, gm, ti.dt))
    corr_o = (af * gm * ti.dt / am) * disc.u_jvp(sto, sto["du"] - sto["v"])
    assert rel_err(R.cpu().numpy(), R_o) < TOL_ASM
    assert rel_err(corr.cpu().numpy(), corr_o) < TOL_ASM
    assert rel_err(gpu_K_scipy(prob, K).toarray(), K_o.toarray()) < TOL_ASM


def test_row_owner_and_element_buffer_tangents_agree():
    """The cube's rows assembled by their owners (16-slot pattern) against the same rows of the cube
    with a disjoint wide-row component appended (32-slot pattern, element buffer): both sum the
    same per-pair values in element order, so they agree to rounding (FMA contraction may differ
    between the two kernels)."""
    out = []
    for with_fan in (False, True):
        mesh, mat, ti = synth.cube_case(3, nu=0.45, n_steps=2) if not with_fan else _asm_case_with_fan(True)
        prob = V.Problem(mesh, mat, "cuda:0")
        print(f"[assembly] {mesh.name} W={prob.slot_width}", flush=True)
        n0 = 64
        st = prob.new_state()
        rs = synth.random_state(n0, 71, {"u": 1e-3})
        rn = synth.random_state(n0, 72, {"u": 1e-3})
        for k in ("u", "p", "v", "du", "dp", "dv"):
            st[k][:n0].copy_(torch.from_numpy(rs[k]))
            st[k + "_n"][:n0].copy_(torch.from_numpy(rn[k]))
        K, R, corr = prob.assemble(st, gpu_ti(ti, 0.3 * ti.dt), V.ASM_RESIDUAL | V.ASM_TANGENT | V.ASM_RKCORR)
        W = prob.slot_width
        rl = prob.host["row_len"][:n0]
        real = np.concatenate([W * i + np.arange(rl[i]) for i in range(n0)])
        blocks = [t.cpu().numpy().reshape(t.shape[0] if t.dim() > 1 else 1, -1)[:, real] for t in (K.A, K.B, K.C, K.D)]
        out.append((R.cpu().numpy()[:n0], corr.cpu().numpy()[:n0], blocks, W))
    (R0, c0, b0, W0), (R1, c1, b1, W1) = out
    assert (W0, W1) == (16, 32)
    assert rel_err(R1, R0) < 1e-14 and rel_err(c1, c0) < 1e-14
    for x, y in zip(b1, b0):
        assert rel_err(x, y) < 1e-14
    same = sum(int(np.array_equal(x, y)) for x, y in zip(b1 + [R1, c1], b0 + [R0, c0]))
    print(f"[assembly] row-owner vs element-buffer: {same} of 6 arrays bitwise equal", flush=True)
