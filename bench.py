"""Benchmark: generalized-alpha Newton steps of the 64^3 cube (nu = 0.499) on one MI355X.

A bench step is one time step of the predictor multi-corrector algorithm
(stage, assemble, scale, nested FGMRES solve, update, per Newton iteration,
until ||R|| / ||R_0|| <= 1e-8) for the synthetic unit-cube compression
workload: 64^3 hexes x 6 Kuhn tets (1,572,864 tets, 274,625 nodes,
1,098,500 unknowns), mu = 1e5, nu = 0.499, rho0 = 1000, dt = 1e-3, top
traction -1e4 ramped over 10 steps.  Timed steps start from rest after the
warm-up steps, so every run does the same work.  Both solver forms run:
FP64 (GMRES at every level) and mixed (FP32 intermediate/inner levels with
CG on the A-solves, FP64 outer FGMRES/Newton); --fp64-a-krylov and
--mixed-a-krylov choose the A-level method of each form.

--workload tube runs the fully incompressible HGO tube (8 x 256 x 160 hexes)
under axial stretch; --workload strip runs the paper's second workload: the eighth of the
10 x 3 x 0.5 mm tensile strip (section 5.2), fully incompressible HGO with
dispersion k_d = 0.226, fibres at +-49.98 deg, symmetry conditions on three
planes, a tensile force ramped to 2 N over 100 s, dt = 1e-5, on the mesh
1/dx = --size (400: 400 x 120 x 20 hexes, 5.76 M tets, 1.02 M nodes).

Prints one JSON line (value = Newton iterations per second of the FP64 form).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Newton-step time & BSR SpMV GB/s (%HBM peak); FP32-inner vs FP64 at 1e-8 rel res"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spmv_A_bytes(n, nnzb, elem):
    """Algorithmic bytes of one 3x3 block SpMV over the nnzb real blocks (the
    padding slots of the fixed-width rows are not counted): values + column
    indices + x (once) + y."""
    return (9 * elem + 4) * nnzb + 2 * 3 * elem * n


def cg_spmv_bytes(n, nnzb, elem):
    """Algorithmic bytes of one CG product launch (w = A z with the direction
    updates p = z + beta p, q = w + beta q): values + column indices of the
    nnzb real blocks, z once, p and q read and written.  The first launch of a
    solve reads no p, q (2 * 3 * elem * n less; about one launch in eight at
    64^3, so the mean is within 0.5 % of this)."""
    return (9 * elem + 4) * nnzb + 5 * 3 * elem * n


def tangent_bytes(n, m, W=16, hgo=False, corr=True):
    """Algorithmic bytes of one row-owner tangent assembly (with the R-bar_k term): each node's
    staged state read once (X, and u, v, v-dot, u-dot at both time levels: 27 doubles; p, p-dot at
    both: 4), its diagonal incidence list and row columns, the tets (and fibres), and the K blocks
    of its W slots (16 doubles each) plus the corr row written once."""
    reads = (31 * 8 + 3 * 4 + W * 4) * n + (16 + 16 + (48 if hgo else 0)) * m
    writes = (16 * 8 * W + (32 if corr else 0)) * n
    return reads, writes


def shat_bytes(n, nnz, elem, idx=4):
    """Algorithmic bytes of one S^ product (the product of the Schur
    preconditioner's CG steps): the real off-diagonal entries (value + column
    index or 2-byte offset), the diagonal, x once (gathers cached) and y."""
    return (elem + idx) * nnz + 3 * elem * n


def shat_idx_bytes(prob):
    return 2 if prob.d.get("shat_off") is not None else 4


# kernel -> (source file, first and end markers of the kernel's source text (None: whole file), summary)
PMC_FILES = {
    "spmv_A": ("linalg.h", None, None, "spmv_A_cube64_pmc.md"),
    "shat": ("solver.hip", "// Off-diagonal part of row ro of S^ times z", "// ---- pipelined CG steps on S^",
             "shat_spmv_cube64_pmc.md"),
    "cg_spmv": ("solver.hip", "// CG iteration j, first half.", "// CG iteration j, second half",
                "cg_spmv_cube64_pmc.md"),
    "assemble_rows": ("assembly.hip", None, None, "assembly_cube64_pmc.md"),
}


def kernel_source_sha(kernel):
    """First 16 hex digits of the SHA-256 of the kernel's source text."""
    import hashlib
    srcname, first, end, _ = PMC_FILES[kernel]
    text = open(os.path.join(ROOT, "paper_1809_06350_amd", "csrc", srcname), "rb").read()
    if first is not None:
        a = text.index(first.encode())
        text = text[a:text.index(end.encode(), a)]
    return hashlib.sha256(text).hexdigest()[:16]


def pmc_traffic(kernel, key):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    that kernel, if its source is unchanged since the counters were taken."""
    prof = os.path.join(ROOT, "profiles", PMC_FILES[kernel][3])
    try:
        sha = kernel_source_sha(kernel)
        kv = dict(line.split(": ", 1) for line in open(prof).read().splitlines() if ": " in line)
        if kv.get("source_sha256_16", "").strip() == sha:
            return float(kv[key])
    except (OSError, ValueError, KeyError):
        pass
    return None


def time_launches(fn, reps=50):
    """Average duration of fn() over reps back-to-back launches between two
    HIP events on the torch current stream (the library's stream)."""
    import torch
    for _ in range(5):
        fn()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps * 1e-3   # seconds per launch


def time_spmv(prob, K, op, x, fp32, reps=50):
    return time_launches(lambda: prob.spmv(K, op, x, fp32), reps)


def shat_real_entries(prob):
    import numpy as np
    n = prob.mesh.n_nodes
    sc = prob.host["shat_col"].reshape(n, -1)
    return int((sc != np.arange(n)[:, None]).sum())


def time_shat(prob, K, fp32, reps=50):
    """The S^ product kernel on the S^ of K: seconds per launch."""
    import torch
    S, Sd, _ = prob.schur_hat(K)
    if fp32:
        S, Sd = S.float(), Sd.float()
    x = torch.randn(prob.mesh.n_nodes, dtype=S.dtype, device=S.device,
                    generator=torch.Generator(S.device).manual_seed(2))
    y = torch.empty_like(x)
    return time_launches(lambda: prob.shat_spmv(S, Sd, x, out=y), reps)


def run_form(prob, mesh, ti, nopts, sopts, steps, warmup, timing=False):
    """Warm-up steps, then `steps` timed steps from rest.  With timing on, every
    launch of the A-block product inside the timed steps is bracketed by HIP
    events on the library's stream (the torch current stream)."""
    import torch
    from paper_1809_06350_amd import vms as V

    import numpy as np
    vm = torch.from_numpy(mesh.dir_mask[:, 0:3].astype(bool)).to(prob.dev)
    dv = torch.from_numpy(np.ascontiguousarray(mesh.dir_vel)).to(prob.dev)

    def from_rest():
        # at rest except for prescribed velocities (the tube's moving end), which hold from t = 0
        st = prob.new_state()
        for key in ("v_n", "du_n"):
            st[key][vm] = dv[vm]
        return st

    K = None
    st = from_rest()
    for s in range(warmup):
        stats, K = prob.step(st, V.time_int(ti.dt, ti.rho_inf, s * ti.dt, ti.n_steps * ti.dt), nopts, sopts, K)
        prob.roll(st)
        log(f"  warmup step {s}: newton={stats['n_newton']} ms={stats['ms_total']:.1f}")
    st = from_rest()
    prob.set_timing(timing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = []
    for s in range(steps):
        stats, K = prob.step(st, V.time_int(ti.dt, ti.rho_inf, s * ti.dt, ti.n_steps * ti.dt), nopts, sopts, K)
        prob.roll(st)
        per.append(stats)
        log(f"  step {s}: newton={stats['n_newton']} outer={stats['it_outer_total']} A={stats['it_A_total']} "
            f"S={stats['it_S_total']} I={stats['it_I_total']} ms={stats['ms_total']:.1f} "
            f"(asm {stats['ms_assemble']:.1f}, solve {stats['ms_solve']:.1f}: scale {stats['ms_scale_total']:.1f} "
            f"setup {stats['ms_setup_total']:.1f} A {stats['ms_A_solve_total']:.1f} S {stats['ms_S_solve_total']:.1f} "
            f"inner {stats['ms_inner_total']:.1f})")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fp32 = sopts.precision == V.MIXED
    ktime = prob.kernel_time(fp32=fp32) if timing else (0.0, 0)
    prob.set_timing(False)
    n_newton = sum(p["n_newton"] for p in per)
    return {"wall_s": wall, "n_newton": n_newton, "per_step": per, "u": st["u"].clone(), "K": K,
            "spmv_A_ms": ktime[0], "spmv_A_launches": ktime[1]}


def time_a_product(prob, ti, nopts, sopts):
    """Duration of the A-level product kernel inside a time step (the plain
    A-block product on GMRES levels, the CG product kernel on CG levels): one
    extra step from rest (after the timed steps) with the library's launch
    timing on, so every working launch records its own start and end with HIP
    events on the library's stream.  Returns (ms in the step, launches)."""
    import torch
    from paper_1809_06350_amd import vms as V
    st = prob.new_state()
    vm = torch.from_numpy(prob.mesh.dir_mask[:, 0:3].astype(bool)).to(prob.dev)
    dv = torch.from_numpy(prob.mesh.dir_vel.copy()).to(prob.dev)
    for key in ("v_n", "du_n"):
        st[key][vm] = dv[vm]
    prob.set_timing(True)
    prob.step(st, V.time_int(ti.dt, ti.rho_inf, 0.0, ti.n_steps * ti.dt), nopts, sopts, None)
    torch.cuda.synchronize()
    ms, cnt = prob.kernel_time(fp32=sopts.precision == V.MIXED)
    prob.set_timing(False)
    return ms, cnt


def cpu_baseline(N=16, nu=0.499, steps=2):
    """The oracle (NumPy/SciPy, sparse LU) on an N^3 sample of the workload:
    its first `steps` time steps from rest, with the BLAS pools held to one
    thread (threadpoolctl), so that the oracle runs on one core.  Returns the
    wall time, the process CPU time over it (the cores actually used) and the
    final state (for the GPU-vs-oracle check at this size)."""
    import synth
    from oracle import assemble as AS
    from oracle import newton as NW
    from threadpoolctl import threadpool_limits
    mesh, mat, ti = synth.cube_case(N, nu=nu, n_steps=10)
    with threadpool_limits(limits=1):
        disc = AS.Discretization(mesh, mat)
        t0, c0 = time.perf_counter(), time.process_time()
        st, n_newton = NW.rest_state(mesh), 0
        for s in range(steps):
            st, info = NW.time_step(disc, ti, st, s * ti.dt, tol_R=1e-8)
            n_newton += info["n_newton"]
        wall, cpu = time.perf_counter() - t0, time.process_time() - c0
    return {"N": N, "wall_s": wall, "cpu_s": cpu, "n_newton": n_newton, "steps": steps,
            "n_unknowns": 4 * mesh.n_nodes, "u": st["u"], "mesh": mesh, "mat": mat, "ti": ti}


def gpu_vs_oracle(cb, nopts, forms):
    """The GPU forms on the oracle's sample (same mesh, steps and Newton tolerance): relative l2 error
    of u after the last step against the oracle's u, per form."""
    import numpy as np
    from paper_1809_06350_amd import vms as V
    mesh, mat, ti = cb["mesh"], cb["mat"], cb["ti"]
    prob = V.Problem(mesh, mat, "cuda:0")
    out = {}
    for name, so in forms.items():
        st, K = prob.new_state(), None
        for s in range(cb["steps"]):
            _, K = prob.step(st, V.time_int(ti.dt, ti.rho_inf, s * ti.dt, ti.n_steps * ti.dt), nopts, so, K)
            prob.roll(st)
        u = st["u"].cpu().numpy()
        out[name] = float(np.linalg.norm(u - cb["u"]) / np.linalg.norm(cb["u"]))
    return out


def time_tangent(prob, ti, reps=20):
    """Wall time per tangent assembly with the R-bar_k term (the step's tangent call) at the predicted
    first state, each call including its host synchronisation (the inverted-element check)."""
    import torch
    from paper_1809_06350_amd import vms as V
    st = prob.new_state()
    tiv = V.time_int(ti.dt, ti.rho_inf, 0.0, ti.n_steps * ti.dt)
    prob.predictor(st, tiv)
    fl = V.ASM_TANGENT | V.ASM_RKCORR
    K, _, corr = prob.assemble(st, tiv, fl)
    for _ in range(3):
        prob.assemble(st, tiv, fl, K=K, corr=corr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        prob.assemble(st, tiv, fl, K=K, corr=corr)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def assemble_only(prob, mesh, ti, reps, hgo):
    """Kernel-level run for hardware counters and the kernel trace: reps tangent assemblies with
    the R-bar_k term (the step's tangent call) at the predicted first state, then the calibration
    copy of spmv_only."""
    import torch
    from paper_1809_06350_amd import vms as V
    st = prob.new_state()
    tiv = V.time_int(ti.dt, ti.rho_inf, 0.0, ti.n_steps * ti.dt)
    prob.predictor(st, tiv)
    fl = V.ASM_TANGENT | V.ASM_RKCORR
    K, _, corr = prob.assemble(st, tiv, fl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        prob.assemble(st, tiv, fl, K=K, corr=corr)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    rd, wr = tangent_bytes(mesh.n_nodes, mesh.n_tets, prob.slot_width, hgo)
    print(json.dumps({"assemble_only": True, "n": mesh.n_nodes, "m": mesh.n_tets, "flags": fl,
                      "bytes_read": rd, "bytes_written": wr, "wall_us_per_call": wall * 1e6,
                      "calibration_bytes_each_way": src.numel() * 8}), flush=True)


def spmv_only(prob, mesh, ti, reps):
    """Kernel-level run for hardware counters: the A-block SpMV (FP64 and FP32)
    on the assembled, scaled first Newton system, and a calibration kernel of
    known traffic: a 1 GiB -> 1 GiB float64 elementwise product (torch), larger
    than the 256 MB Infinity Cache, so that each dispatch reads and writes
    2^30 bytes of HBM."""
    import torch
    from paper_1809_06350_amd import vms as V
    st = prob.new_state()
    tiv = V.time_int(ti.dt, ti.rho_inf, 0.0, ti.n_steps * ti.dt)
    prob.predictor(st, tiv)
    K, R, _ = prob.assemble(st, tiv, V.ASM_RESIDUAL | V.ASM_TANGENT)
    K32 = prob.new_matrix(mirror32=True)
    for a, b in ((K32.A, K.A), (K32.B, K.B), (K32.C, K.C), (K32.D, K.D)):
        a.copy_(b)
    prob.prepare(K32, R, None, 1e-15, True)
    n = mesh.n_nodes
    x = torch.randn(n, 3, dtype=torch.float64, device="cuda:0", generator=torch.Generator("cuda:0").manual_seed(1))
    xf = x.float()
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        prob.spmv(K32, V.OP_A, x, False)
    for _ in range(reps):
        prob.spmv(K32, V.OP_A, xf, True)
    S, Sd, _ = prob.schur_hat(K32)
    S32, Sd32 = S.float(), Sd.float()
    xs = torch.randn(n, dtype=torch.float64, device="cuda:0", generator=torch.Generator("cuda:0").manual_seed(2))
    ys, xs32 = torch.empty_like(xs), xs.float()
    ys32 = torch.empty_like(xs32)
    for _ in range(reps):
        prob.shat_spmv(S, Sd, xs, out=ys)
    for _ in range(reps):
        prob.shat_spmv(S32, Sd32, xs32, out=ys32)
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    t64 = time_spmv(prob, K32, V.OP_A, x, False)
    t32 = time_spmv(prob, K32, V.OP_A, xf, True)
    # the HBM rate a plain streaming kernel reaches on this device (context for the roofline fractions)
    tcal = time_launches(lambda: torch.mul(src, 1.0, out=dst))
    acc = torch.empty(1, dtype=torch.float64, device="cuda:0")
    tsum = time_launches(lambda: torch.sum(src, dim=0, out=acc[0]))
    nzs = shat_real_entries(prob)
    nz = int(prob.host["row_len"].sum())
    print(json.dumps({"spmv_only": True, "n": n, "nnzb": nz, "nnzb_slots": prob.nnzb,
                      "calibration_bytes_each_way": src.numel() * 8,
                      "calibration_us": tcal * 1e6, "copy_GBps": 2 * src.numel() * 8 / tcal / 1e9,
                      "read_only_sum_us": tsum * 1e6, "read_only_GBps": src.numel() * 8 / tsum / 1e9,
                      "bytes_fp64": spmv_A_bytes(n, nz, 8), "us_fp64": t64 * 1e6,
                      "bytes_fp32": spmv_A_bytes(n, nz, 4), "us_fp32": t32 * 1e6,
                      "shat_nnz": nzs, "shat_bytes_fp64": shat_bytes(n, nzs, 8, shat_idx_bytes(prob)),
                      "shat_us_fp64": time_shat(prob, K32, False) * 1e6,
                      "shat_bytes_fp32": shat_bytes(n, nzs, 4, shat_idx_bytes(prob)),
                      "shat_us_fp32": time_shat(prob, K32, True) * 1e6}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube", choices=["cube", "strip", "tube"],
                    help="cube: the unit-cube compression (the headline); strip: the eighth of the anisotropic "
                         "tensile strip of section 5.2 (HGO with dispersion, symmetry conditions, dt = 1e-5); "
                         "tube: the fully incompressible HGO tube under axial stretch (8 x 256 x 160 hexes)")
    ap.add_argument("--size", type=int, default=None,
                    help="cube: hexes per edge (64); strip: 1/dx of the half-length (400: 400 x 120 x 20 hexes); "
                         "tube: hexes around the circumference (256; radial and axial counts scale with it)")
    ap.add_argument("--stretch", type=float, default=1.5,
                    help="tube: axial stretch reached after the 20-step ramp")
    ap.add_argument("--dir-lift", default="auto", choices=["auto", "on", "off"],
                    help="Dirichlet velocity components in the predictor: lifted (the prescribed motion enters "
                         "through R-bar_k in the first corrector) or preset; auto = lifted for the tube")
    ap.add_argument("--nu", type=float, default=0.499)
    ap.add_argument("--kd", type=float, default=0.226, help="strip: fibre dispersion k_d")
    ap.add_argument("--fibre-deg", type=float, default=49.98,
                    help="strip: fibre angle to the loading direction (49.98 circumferential, 40.02 axial)")
    ap.add_argument("--dt", type=float, default=None, help="time step (cube 1e-3, strip 1e-5)")
    ap.add_argument("--tol-abs", type=float, default=None,
                    help="absolute Newton tolerance beside the relative 1e-8 (cube: none; strip: 1e-15, which "
                         "ends the first step from rest, whose initial residual is ~1e-9 against a round-off "
                         "floor near 2e-17)")
    ap.add_argument("--forms", default="fp64,mixed")
    ap.add_argument("--shat-degree", type=int, default=16)
    ap.add_argument("--shat-ratio", type=float, default=20.0)
    ap.add_argument("--a-prec", default="auto", choices=["auto", "bj", "amg"],
                    help="preconditioner of the A-levels: 3x3 block-Jacobi or the aggregation multigrid; auto = "
                         "block-Jacobi on the cube (mass-dominated A at dt = 1e-3), multigrid on the strip and tube")
    ap.add_argument("--amg-levels", type=int, default=3)
    ap.add_argument("--amg-coarse-degree", type=int, default=None,
                    help="Chebyshev degree of the multigrid's coarsest-level smoothing; default 4 on the tube "
                         "(15 %% less time per step than 2; 8 and 16 are slower again), 2 elsewhere (4 and 8 "
                         "change nothing on the strip)")
    ap.add_argument("--amg-mid-degree", type=int, default=None,
                    help="Chebyshev degree of the multigrid's middle level (between the finest and the coarsest); "
                         "default 4 on the tube (6 %% less time per step than the finest level's 2), 0 = the "
                         "finest level's degree elsewhere (4 is slower on the strip)")
    ap.add_argument("--amg-degree", type=int, default=None,
                    help="Chebyshev degree of the multigrid's pre- and post-smoothing; default 3 on the strip "
                         "(5-7 %% less time per step than 2), 2 elsewhere (the tube's steps take more outer "
                         "iterations with 3)")
    ap.add_argument("--shat-method", default=None, choices=["chebyshev", "cg", "none"],
                    help="S^ preconditioner of the Schur solve: Chebyshev polynomial or CG steps (--shat-degree)")
    ap.add_argument("--outer-tol", type=float, default=1e-8,
                    help="relative tolerance of the outer FGMRES (the Newton tolerance stays 1e-8)")
    ap.add_argument("--fp64-tol", default="5e-5,1.5e-5,7e-5",
                    help="intermediate A, Schur and inner tolerances of the FP64 form")
    ap.add_argument("--mixed-tol", default="5e-5,1.5e-5,7e-5",
                    help="intermediate A, Schur and inner tolerances of the mixed form")
    ap.add_argument("--orth", default="cgs1", choices=["cgs2", "cgs1", "cgs_ifneeded", "mgs"],
                    help="Arnoldi orthogonalisation of every Krylov level")
    akc = ["gmres", "cg-inner", "cg", "cg-inner-sym", "cg-sym"]
    ap.add_argument("--fp64-a-krylov", default=None, choices=akc,
                    help="Krylov method of the A-solves in the FP64 form: GMRES, or CG at the inner level or at "
                         "both A-levels, on A itself or on (A + A^T)/2 (-sym); default gmres for the cube, cg for "
                         "the strip (about 190 iterations per A-solve, where GMRES's growing orthogonalisation "
                         "costs twice the time)")
    ap.add_argument("--mixed-a-krylov", default="cg", choices=akc,
                    help="the same for the mixed form")
    ap.add_argument("--precond", default="ldu", choices=["ldu", "upper", "lower", "diag", "simple"],
                    help="block preconditioner: the nested Schur complement reduction (ldu) and its partial "
                         "factorizations, or SIMPLE")
    ap.add_argument("--schur-step", default="krylov", choices=["krylov", "shat"],
                    help="Schur step: Krylov solve to the Schur tolerance, or one S^ preconditioner application")
    ap.add_argument("--relax-inner", default="off", choices=["on", "off"],
                    help="relax the inner tolerance of the Schur products as the Schur level converges "
                         "(relax_inner; off, as in the paper, by default)")
    ap.add_argument("--schur-mass", type=float, default=None,
                    help="weight of the lumped pressure-mass term in the Schur preconditioner (schur_mass; 0: off); "
                         "default 1 on the tube (with --shat-method none there: a stiffness-dominated A at dt = "
                         "0.05 makes S close to a scaled pressure mass matrix) and on the strip (beside the CG "
                         "steps on S^: 28 %% less time per step at 1/dx = 400), 0 on the cube")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-timing", action="store_true",
                    help="also event-time every A-block product launch inside the timed steps (each launch then "
                         "carries start/stop events, which lengthens it and the steps by the event overhead)")
    ap.add_argument("--spmv-only", type=int, default=0,
                    help="only launch the A-block SpMV (FP64 and FP32) this many times each on the first "
                         "Newton system, plus a 256 MiB device copy as the counter calibration kernel")
    ap.add_argument("--assemble-only", type=int, default=0,
                    help="only run the tangent assembly (with the R-bar_k term) this many times at the first "
                         "predicted state, plus the copy calibration kernel (for the kernel trace and counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1809_06350_amd import vms as V

    cube = args.workload == "cube"
    N = args.size or {"cube": 64, "strip": 400, "tube": 256}[args.workload]
    tube = args.workload == "tube"
    if args.schur_mass is None:
        args.schur_mass = 0.0 if cube else 1.0
    if args.shat_method is None:
        args.shat_method = "none" if tube and args.schur_mass > 0.0 else "cg"
    if args.amg_degree is None:
        args.amg_degree = 3 if args.workload == "strip" else 2
    if args.amg_coarse_degree is None:
        args.amg_coarse_degree = 4 if args.workload == "tube" else 2
    if args.amg_mid_degree is None:
        args.amg_mid_degree = 4 if args.workload == "tube" else 0
    if args.a_prec == "auto":
        args.a_prec = "bj" if args.workload == "cube" else "amg"
    if args.workload == "tube":
        dt = args.dt or 0.05
        nt = N
        nr, nz = max(1, nt // 32), max(1, (nt * 5) // 8)
        mesh, mat, ti = synth.tube_case(nr, nt, nz, dt=dt, n_steps=20, stretch=args.stretch)
        wl = (f"HGO tube {nr}x{nt}x{nz} hexes x 6 Kuhn tets, fully incompressible, fibres +-45 deg, axial stretch "
              f"{args.stretch} over 20 steps, dt={dt:g}, Newton 1e-8, FGMRES {args.outer_tol:g}")
        args.no_cpu_baseline = True
    elif cube:
        dt = args.dt or 1e-3
        mesh, mat, ti = synth.cube_case(N, nu=args.nu, n_steps=10, dt=dt)
        wl = f"cube{N}^3 Kuhn tets, nu={args.nu}, neo-Hookean, dt={dt:g}, Newton 1e-8, FGMRES {args.outer_tol:g}"
    else:
        dt = args.dt or 1e-5
        mesh, mat, ti = synth.strip_case(N, kd=args.kd, fibre_deg=args.fibre_deg, dt=dt)
        nx, ny, nz = synth.strip_dims(N)
        wl = (f"tensile strip (eighth) 1/dx={N}: {nx}x{ny}x{nz} hexes x 6 Kuhn tets, incompressible HGO "
              f"k_d={args.kd}, phi={args.fibre_deg} deg, 2 N over 100 s, dt={dt:g}, Newton 1e-8, "
              f"FGMRES {args.outer_tol:g} "
              f"(Newton also ends below {args.tol_abs if args.tol_abs is not None else 1e-15:g} absolute)")
        args.no_cpu_baseline = True
    log(f"{mesh.name}: nodes={mesh.n_nodes} tets={mesh.n_tets}")
    prob = V.Problem(mesh, mat, "cuda:0")
    if mesh.fibre is not None:
        prob.set_fibres(*synth.fibre_field(mesh, mesh.meta["fibre_rad"]))
    amg_info = None
    if args.a_prec == "amg":
        t0 = time.perf_counter()
        amg_info = prob.setup_amg(V.amg_opts(max_levels=args.amg_levels, degree=args.amg_degree,
                                             coarse_degree=args.amg_coarse_degree,
                                             mid_degree=args.amg_mid_degree))
        amg_info["host_setup_s"] = time.perf_counter() - t0
        amg_info["degrees"] = {"finest": args.amg_degree, "middle": args.amg_mid_degree or args.amg_degree,
                               "coarsest": args.amg_coarse_degree}
        log(f"multigrid: levels {amg_info['n']} ({amg_info['host_setup_s']:.2f} s host set-up)")
    apc = V.APC_AMG if args.a_prec == "amg" else V.APC_BJ
    n, nnzb = mesh.n_nodes, int(prob.host["row_len"].sum())   # real blocks (slots: prob.nnzb)
    tol_abs = args.tol_abs if args.tol_abs is not None else (1e-50 if cube else 1e-15)
    lift = {"on": 1, "off": 0}.get(args.dir_lift, 1 if args.workload == "tube" else 0)
    nopts = V.newton_opts(tol_R=1e-8, tol_A=tol_abs, l_max=20, dir_lift=lift)
    mt = [float(x) for x in args.mixed_tol.split(",")]
    ft = [float(x) for x in args.fp64_tol.split(",")]
    if args.spmv_only:
        spmv_only(prob, mesh, ti, args.spmv_only)
        return
    if args.assemble_only:
        assemble_only(prob, mesh, ti, args.assemble_only, mesh.fibre is not None)
        return
    orth = {"cgs2": V.ORTH_CGS2, "cgs1": V.ORTH_CGS1, "cgs_ifneeded": V.ORTH_CGS_IFNEEDED,
            "mgs": V.ORTH_MGS}[args.orth]
    akm = {"gmres": (V.AK_GMRES, 0), "cg-inner": (V.AK_CG_INNER, 0), "cg": (V.AK_CG, 0),
           "cg-inner-sym": (V.AK_CG_INNER, 1), "cg-sym": (V.AK_CG, 1)}
    if args.fp64_a_krylov is None:
        args.fp64_a_krylov = "gmres" if cube else "cg"   # many A-iterations per solve off the cube
    relax = int(args.relax_inner == "on")
    fk, fs = akm[args.fp64_a_krylov]
    mk, ms = akm[args.mixed_a_krylov]
    sm = {"chebyshev": V.SHAT_CHEBYSHEV, "cg": V.SHAT_CG, "none": V.SHAT_NONE}[args.shat_method]
    pc = {"ldu": V.PC_LDU, "upper": V.PC_UPPER, "lower": V.PC_LOWER, "diag": V.PC_DIAG,
          "simple": V.PC_SIMPLE}[args.precond]
    ss = {"krylov": V.SCHUR_KRYLOV, "shat": V.SCHUR_SHAT}[args.schur_step]
    forms = {
        "fp64": V.solver_opts(rtol=args.outer_tol, rtol_A=ft[0], rtol_S=ft[1], rtol_I=ft[2], shat_degree=args.shat_degree,
                              shat_ratio=args.shat_ratio, orth=orth, a_krylov=fk, cg_symmetrise=fs,
                              shat_method=sm, precond=pc, schur_solve=ss, relax_inner=relax,
                              schur_mass=args.schur_mass, a_prec=apc),
        "mixed": V.solver_opts(rtol=args.outer_tol, rtol_A=mt[0], rtol_S=mt[1], rtol_I=mt[2], precision=V.MIXED,
                               shat_degree=args.shat_degree, shat_ratio=args.shat_ratio, orth=orth, a_krylov=mk,
                               cg_symmetrise=ms, shat_method=sm, precond=pc, schur_solve=ss, relax_inner=relax,
                               schur_mass=args.schur_mass, a_prec=apc),
    }
    results = {}
    for name in args.forms.split(","):
        log(f"form {name}")
        results[name] = run_form(prob, mesh, ti, nopts, forms[name], args.steps, args.warmup,
                                 timing=args.kernel_timing)

    primary = "fp64" if "fp64" in results else list(results)[0]
    r = results[primary]
    value = r["n_newton"] / r["wall_s"]

    # dominant kernel of the FP64 form: the A-level product (the plain A-block product on GMRES levels,
    # the CG product kernel that fuses it with the direction updates on CG levels) or the S^ product of
    # the Schur preconditioner's CG steps, whichever takes more time per step.  The A-level product is
    # timed inside one extra time step from rest: every working launch records its own start and end
    # (launches and ms per step counted directly; back-to-back launches of the plain product run
    # faster, about 55 against 62 us at 64^3, on caches that the steps do not leave warm).  The S^
    # product is timed as the average over 50 back-to-back launches on the S^ of the workload's last
    # Newton system, between two HIP events on the library's stream (the torch current stream), times
    # the launches the solver statistics give (the kernel trace of the steps gives the same duration).
    # With --kernel-timing every A-product launch inside the timed steps is event-timed as well and
    # reported beside it (that figure includes the per-launch event overhead).
    K = r["K"]
    so = forms[primary]
    x64 = torch.randn(n, 3, dtype=torch.float64, device="cuda:0", generator=torch.Generator("cuda:0").manual_seed(1))
    t64 = time_spmv(prob, K, V.OP_A, x64, False)
    by64 = spmv_A_bytes(n, nnzb, 8)
    nzs = shat_real_entries(prob)
    ts64 = time_shat(prob, K, False)
    bys64 = shat_bytes(n, nzs, 8, shat_idx_bytes(prob))
    steps_stats = r["per_step"]
    # the CG steps on S^: one product to start and one per step
    launches_S = (sum(p["it_S_total"] for p in steps_stats) / args.steps * (so.shat_degree + 1)
                  if so.shat_method == V.SHAT_CG else 0.0)
    isolated = "HIP events around 50 back-to-back launches on the last Newton system of the timed steps"
    in_step = ("HIP events recorded by each working launch of the kernel (hipExtLaunchKernelGGL, the library's "
               "stream) during one extra time step from rest after the timed steps")
    kern = {
        "k_shat_spmv<double>": {"achieved": bys64 / ts64 / 1e9, "us_per_launch": ts64 * 1e6,
                               "bytes_per_launch": bys64, "launches_per_step": launches_S,
                               "est_ms_per_step": launches_S * ts64 * 1e3,
                               "traffic": pmc_traffic("shat", "traffic_bytes_fp64") if cube and N == 64 else None,
                               "timing": isolated},
    }
    # the A-level product runs as the plain A-block product on GMRES levels and inside the CG product
    # kernel on CG levels; with one method at both levels it is timed inside a time step
    if so.a_krylov in (V.AK_GMRES, V.AK_CG):
        cg_levels = so.a_krylov == V.AK_CG
        ms_a, cnt_a = time_a_product(prob, ti, nopts, so)
        ta = ms_a * 1e-3 / max(cnt_a, 1)
        bya = cg_spmv_bytes(n, nnzb, 8) if cg_levels else by64
        name = "k_cg_spmv<double>" if cg_levels else "k_spmv_A<double,double>"
        kern[name] = {"achieved": bya / ta / 1e9, "us_per_launch": ta * 1e6, "bytes_per_launch": bya,
                      "launches_per_step": cnt_a, "est_ms_per_step": ms_a,
                      "traffic": (pmc_traffic("cg_spmv" if cg_levels else "spmv_A", "traffic_bytes_fp64")
                                  if cube and N == 64 else None),
                      "timing": in_step}
        if not cg_levels:
            kern[name]["back_to_back_us_per_launch"] = t64 * 1e6
    else:
        launches_A = sum(p["it_A_total"] for p in steps_stats) / args.steps
        kern["k_spmv_A<double,double>"] = {
            "achieved": by64 / t64 / 1e9, "us_per_launch": t64 * 1e6, "bytes_per_launch": by64,
            "launches_per_step": launches_A, "est_ms_per_step": launches_A * t64 * 1e3,
            "traffic": pmc_traffic("spmv_A", "traffic_bytes_fp64") if cube and N == 64 else None,
            "timing": isolated}
    dom = max(kern, key=lambda k: kern[k]["est_ms_per_step"])
    kd = kern[dom]
    roof = {"bound": "hbm", "kernel": dom, "achieved": kd["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": kd["achieved"] / HBM_PEAK_GBS, "traffic": kd["traffic"],
            "bytes_per_launch": kd["bytes_per_launch"], "us_per_launch": kd["us_per_launch"],
            "timing": kd["timing"]}
    if amg_info is not None:
        roof["scope"] = ("the dominant kernel among the products the bench times (A-level and S^ products); with the "
                         "multigrid on, its finest-level smoothing and residual kernels (k_amgf_*) take more of the "
                         "step than the CG product (see the kernel trace of this workload)")
    # context: the rate of a plain streaming kernel on this device (1 GiB -> 1 GiB float64 copy-scale,
    # larger than the Infinity Cache), and the dominant kernel's measured HBM traffic per launch over
    # its duration against it
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    tcopy = time_launches(lambda: torch.mul(src, 1.0, out=dst))
    roof["copy_GBps"] = 2 * src.numel() * 8 / tcopy / 1e9
    if kd["traffic"]:
        roof["traffic_GBps"] = kd["traffic"] / (kd["us_per_launch"] * 1e-6) / 1e9
        roof["traffic_frac_of_copy"] = roof["traffic_GBps"] / roof["copy_GBps"]
    del src, dst
    extra = {"fp64_kernels": kern}
    if r["spmv_A_launches"] > 0:
        t_in = r["spmv_A_ms"] * 1e-3 / r["spmv_A_launches"]
        by_in = cg_spmv_bytes(n, nnzb, 8) if so.a_krylov == V.AK_CG else by64
        extra["spmv_A_in_steps"] = {"us_per_launch": t_in * 1e6, "GB/s": by_in / t_in / 1e9,
                                    "launches": r["spmv_A_launches"],
                                    "note": "start/stop events of every working launch in the timed steps"}
    ttan = time_tangent(prob, ti)
    rd, wr = tangent_bytes(n, mesh.n_tets, prob.slot_width, mesh.fibre is not None)
    extra["tangent_assembly"] = {"us_per_call": ttan * 1e6, "bytes_read": rd, "bytes_written": wr,
                                 "GB/s": (rd + wr) / ttan / 1e9, "frac_hbm": (rd + wr) / ttan / 1e9 / HBM_PEAK_GBS,
                                 "traffic": (pmc_traffic("assemble_rows", "traffic_bytes")
                                             if cube and N == 64 else None),
                                 "timing": "wall time per call over 20 calls, each with its host synchronisation"}
    first = r["per_step"][0]
    extra["first_step"] = {"ms": first["ms_total"], "n_newton": first["n_newton"],
                           "ms_per_newton": first["ms_total"] / max(first["n_newton"], 1)}
    if "mixed" in results:
        rm = results["mixed"]
        by32 = spmv_A_bytes(n, nnzb, 4)
        t32 = time_spmv(prob, rm["K"], V.OP_A, x64.float(), True)
        extra["spmv_A_fp32"] = {"GB/s": by32 / t32 / 1e9, "us_per_launch": t32 * 1e6, "bytes_per_launch": by32,
                                "frac_hbm": by32 / t32 / 1e9 / HBM_PEAK_GBS,
                                "traffic": pmc_traffic("spmv_A", "traffic_bytes_fp32") if cube and N == 64 else None}
        ts32 = time_shat(prob, rm["K"], True)
        bys32 = shat_bytes(n, nzs, 4, shat_idx_bytes(prob))
        extra["shat_fp32"] = {"GB/s": bys32 / ts32 / 1e9, "us_per_launch": ts32 * 1e6, "bytes_per_launch": bys32,
                              "frac_hbm": bys32 / ts32 / 1e9 / HBM_PEAK_GBS,
                              "traffic": pmc_traffic("shat", "traffic_bytes_fp32") if cube and N == 64 else None}
        u64 = results.get("fp64", rm)["u"]
        err = float((rm["u"] - u64).norm() / u64.norm()) if "fp64" in results else None
        extra["mixed"] = {"newton_per_s": rm["n_newton"] / rm["wall_s"],
                          "ms_per_newton": 1e3 * rm["wall_s"] / rm["n_newton"],
                          "ms_per_step": 1e3 * rm["wall_s"] / args.steps,
                          "first_step_ms": rm["per_step"][0]["ms_total"],
                          "speedup_vs_fp64": (r["wall_s"] / rm["wall_s"]) if "fp64" in results else None,
                          "u_rel_err_vs_fp64": err}
    phase_keys = ("ms_scale_total", "ms_setup_total", "ms_outer_total", "ms_A_solve_total", "ms_S_solve_total",
                  "ms_inner_total")
    for name, rr in results.items():
        last = rr["per_step"][-1]
        extra[f"{name}_last_step"] = {k: last[k] for k in ("n_newton", "it_outer_total", "it_A_total", "it_S_total",
                                                           "it_I_total", "ms_assemble", "ms_solve", "ms_total")}
        # device time per step of the solver's phases (HIP events on the library's stream), mean over the
        # timed steps; they nest: outer includes A and S, S includes inner
        per = rr["per_step"]
        ph = {k[3:-6]: sum(p[k] for p in per) / len(per) for k in phase_keys}
        ph["outer_excl"] = ph["outer"] - ph["A_solve"] - ph["S_solve"]
        ph["S_excl"] = ph["S_solve"] - ph["inner"]
        ph["assemble_host"] = sum(p["ms_assemble"] for p in per) / len(per)
        extra[f"{name}_phase_ms_per_step"] = ph
    out = {"metric": METRIC, "value": value, "unit": "newton_steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * r["wall_s"] / args.steps,
           "ms_per_newton_step": 1e3 * r["wall_s"] / r["n_newton"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64" if primary == "fp64" else "f32+f64",
           "data": "synthetic",
           "config": {"workload": wl,
                      "nodes": n, "tets": mesh.n_tets, "unknowns": 4 * n, "nnzb": nnzb,
                      "block_slots": prob.nnzb,
                      "shat_degree": args.shat_degree, "shat_ratio": args.shat_ratio,
                      "shat_method": args.shat_method, "orth": args.orth, "precond": args.precond,
                      "schur_step": args.schur_step,
                      "tolerances": {"outer": args.outer_tol, "fp64_A_S_I": ft, "mixed_A_S_I": mt,
                                     "relax_inner": relax, "schur_mass": args.schur_mass},
                      "a_prec": args.a_prec, "amg": amg_info,
                      "a_krylov": {"fp64": args.fp64_a_krylov, "mixed": args.mixed_a_krylov},
                      "parallelism": "single GPU"},
           "roofline": roof}
    out.update(extra)
    if not args.no_cpu_baseline:
        # the oracle on two samples of the workload (12^3 and 16^3 cubes, 2 time steps each); its time per
        # Newton iteration is fitted as c * unknowns^alpha through the two points and evaluated at the
        # workload's size (sparse LU grows faster than linearly, so a linear scaling would flatter the CPU)
        import math
        pts = []
        for Ns in (12, 16):
            log(f"cpu baseline: oracle on the {Ns}^3 sample")
            pts.append(cpu_baseline(Ns, args.nu))
        t_per = [p["wall_s"] / p["n_newton"] for p in pts]
        alpha = math.log(t_per[1] / t_per[0]) / math.log(pts[1]["n_unknowns"] / pts[0]["n_unknowns"])
        t_full = t_per[1] * (4 * n / pts[1]["n_unknowns"]) ** alpha
        cores = sum(p["cpu_s"] for p in pts) / sum(p["wall_s"] for p in pts)
        out["cpu_baseline"] = {
            "value": 1.0 / t_full, "unit": "newton_steps/s", "cores": round(cores, 2), "kind": "oracle",
            "sample": (f"the first 2 time steps of the 12^3 and 16^3 cubes (nu={args.nu}), timed on the host "
                       f"with the BLAS pools held to 1 thread; seconds per Newton iteration "
                       + ", ".join(f"{p['N']}^3 ({p['n_unknowns']} unknowns): {t:.3f} s ({p['n_newton']} its)"
                                   for p, t in zip(pts, t_per))
                       + f"; fitted t ~ unknowns^{alpha:.2f}, evaluated at {4 * n} unknowns; cores = process "
                         f"CPU time / wall time; host os.cpu_count()={os.cpu_count()}, "
                         f"OMP_NUM_THREADS={os.environ.get('OMP_NUM_THREADS', 'unset')}"),
            "points": [{"N": p["N"], "unknowns": p["n_unknowns"], "s_per_newton": t, "newton": p["n_newton"],
                        "wall_s": p["wall_s"], "cpu_s": p["cpu_s"]} for p, t in zip(pts, t_per)],
            "fitted_exponent": alpha}
        if cube:
            log("oracle check: the GPU forms on the 16^3 sample")
            out["oracle_check_16"] = {
                "u_rel_err": gpu_vs_oracle(pts[1], nopts, {k: forms[k] for k in results}),
                "note": "GPU u after the sample's 2 time steps (bench tolerances, Newton 1e-8) against the "
                        "oracle's (sparse LU, Newton 1e-8), relative l2"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
