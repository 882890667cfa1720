"""vms_step_noalloc (the time step whose workspace is the library's static
device scratch) against vms_step with a caller workspace: two calls in a row
on one device, the second on a smaller mesh, each compared with the ordinary
entry point on the same inputs; then a mesh too large for the scratch is
refused before anything is launched."""
import numpy as np
import pytest
import torch

import synth
from paper_1809_06350_amd import vms as V

pytestmark = pytest.mark.gpu

KEYS = ("u", "p", "v", "du", "dp", "dv")


def _steps(N, noalloc, nsteps, precision):
    mesh, mat, ti = synth.cube_case(N, nu=0.45, n_steps=4)
    prob = V.Problem(mesh, mat, "cuda:0")
    st = prob.new_state()
    if precision == V.MIXED:
        # FP32 intermediate and inner levels: the benchmark's tolerances (the FP32 floor is near 1e-7)
        nopts = V.newton_opts(tol_R=1e-8)
        sopts = V.solver_opts(rtol=1e-8, precision=V.MIXED, a_krylov=V.AK_CG)
    else:
        nopts = V.newton_opts(tol_R=1e-10)
        sopts = V.solver_opts(rtol=1e-10, rtol_A=1e-10, rtol_S=1e-10, rtol_I=1e-12)
    K, out = None, []
    for s in range(nsteps):
        tiv = V.time_int(ti.dt, ti.rho_inf, s * ti.dt, ti.n_steps * ti.dt)
        fn = prob.step_noalloc if noalloc else prob.step
        stats, K = fn(st, tiv, nopts, sopts, K)
        assert stats["status"] == 0 and stats["n_newton"] >= 1
        out.append({k: st[k].cpu().numpy().copy() for k in KEYS})
        prob.roll(st)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("precision", [V.FP64, V.MIXED])
def test_noalloc_step_matches_step_twice_then_smaller(precision):
    for N in (6, 4):
        print(f"[noalloc] cube {N}^3 precision={precision}", flush=True)
        ref = _steps(N, False, 2, precision)
        got = _steps(N, True, 2, precision)
        for s in range(2):
            for k in KEYS:
                scale = np.abs(ref[s][k]).max()
                assert np.abs(got[s][k] - ref[s][k]).max() <= 1e-12 * scale, (N, s, k)


def test_noalloc_refuses_a_mesh_larger_than_the_scratch():
    mesh, mat, ti = synth.cube_case(12, nu=0.45)
    prob = V.Problem(mesh, mat, "cuda:0")
    st = prob.new_state()
    with pytest.raises(V.VmsError) as e:
        prob.step_noalloc(st, V.time_int(ti.dt, ti.rho_inf, 0.0, ti.dt), V.newton_opts(), V.solver_opts())
    assert e.value.code == -3
    assert float(st["u"].abs().max()) == 0.0
