"""Pins of the oracle's generalized-alpha parameters and load timing (section 3.2).

The parameters alpha_m, alpha_f, gamma of ``oracle.element.genalpha`` are
checked against what section 3.2 fixes about them, not against the formula
itself:

* literal values at rho_inf = 0.5 (the paper's choice) and rho_inf = 1;
* applied to the scalar first-order model problem y' = lambda y through the
  scheme's own recurrences (the y_{n+1} update and the two stage
  definitions), both roots of the amplification matrix tend to rho_inf in
  modulus as lambda dt -> -infinity (the spectral radius at the highest mode);
* the scheme is second-order accurate (errors fall about 4x per halving of dt).

Each check is also run with one parameter perturbed by 5 %, and at least one
check must then fail, so that a wrong alpha_m, alpha_f or gamma cannot pass.

The dead load is evaluated at t_{n+alpha_f}, the time level of the stage at
which the residual is evaluated.  That is pinned by the whole oracle time
step: on a small cube under a linearly ramped traction, u(T) converges at
second order in dt against a fine-step run, while the same integrator with the
load taken at t_{n+1} drops to first order.
"""
import numpy as np
import pytest

import synth
from oracle import assemble as AS
from oracle import element as E
from oracle import newton as NW


def amplification(am, af, gm, z):
    """Amplification matrix of (y, dt y') for y' = lambda y, z = lambda dt:
    y'_n + am (y'_{n+1} - y'_n) = lambda (y_n + af (y_{n+1} - y_n)) and
    y_{n+1} = y_n + dt y'_n + gm dt (y'_{n+1} - y'_n)."""
    lhs = np.array([[-z * af, am], [1.0, -gm]], dtype=complex)
    rhs = np.array([[z * (1.0 - af), -(1.0 - am)], [1.0, 1.0 - gm]], dtype=complex)
    return np.linalg.solve(lhs, rhs)


def integrate(am, af, gm, lam, T, N):
    """y(T) of y' = lambda y, y(0) = 1, y'(0) = lambda, in N generalized-alpha steps."""
    dt = T / N
    M = amplification(am, af, gm, lam * dt)
    x = np.array([1.0, lam * dt], dtype=complex)   # (y, dt y')
    for _ in range(N):
        x = M @ x
    return x[0]


def spectral_radius_at_infinity(am, af, gm):
    return float(np.abs(np.linalg.eigvals(amplification(am, af, gm, -1.0e10))).max())


def convergence_ratios(am, af, gm):
    lam = -1.0 + 4.0j
    errs = [abs(integrate(am, af, gm, lam, 1.0, N) - np.exp(lam)) for N in (40, 80, 160)]
    return [errs[0] / errs[1], errs[1] / errs[2]]


def failures(params, rho_inf):
    am, af, gm = params
    out = []
    if abs(spectral_radius_at_infinity(am, af, gm) - rho_inf) > 1e-4:
        out.append("rho_inf")
    if min(convergence_ratios(am, af, gm)) < 3.5:
        out.append("order")
    return out


def test_literal_values():
    am, af, gm = E.genalpha(0.5)
    assert am == pytest.approx(5.0 / 6.0, abs=1e-15)
    assert af == pytest.approx(2.0 / 3.0, abs=1e-15)
    assert gm == pytest.approx(2.0 / 3.0, abs=1e-15)
    assert E.genalpha(1.0) == pytest.approx((0.5, 0.5, 0.5), abs=1e-15)
    assert E.genalpha(0.0) == pytest.approx((1.5, 1.0, 1.0), abs=1e-15)


@pytest.mark.parametrize("rho_inf", [0.0, 0.5, 1.0])
def test_spectral_radius_and_second_order(rho_inf):
    assert failures(E.genalpha(rho_inf), rho_inf) == []


@pytest.mark.parametrize("which", [0, 1, 2])
@pytest.mark.parametrize("rho_inf", [0.5, 1.0])
def test_a_perturbed_parameter_is_caught(rho_inf, which):
    p = list(E.genalpha(rho_inf))
    p[which] *= 1.05
    assert failures(tuple(p), rho_inf) != []


def _ramped_cube_u(N, T, load_shift=0.0):
    """u at T after N oracle steps of the 2^3 cube (nu = 0.3) from rest under a
    traction ramped to full at T; load_shift moves the load's evaluation time
    by load_shift * dt (a planted mistake when nonzero)."""
    mesh, mat, ti = synth.cube_case(2, nu=0.3, dt=T / N, n_steps=N)
    disc = AS.Discretization(mesh, mat)
    st = NW.rest_state(mesh)
    orig = NW.load_scale
    if load_shift:
        NW.load_scale = lambda ti_, t: orig(ti_, t + load_shift * ti_.dt)
    try:
        for s in range(N):
            st, info = NW.time_step(disc, ti, st, s * ti.dt, tol_R=1e-12)
            assert info["converged"]
    finally:
        NW.load_scale = orig
    return st["u"]


def test_load_at_alpha_f_stage_gives_second_order():
    T = 0.05
    ref = _ramped_cube_u(64, T)

    def ratio(shift):
        e = [np.linalg.norm(_ramped_cube_u(N, T, shift) - ref) for N in (8, 16)]
        return e[0] / e[1]

    assert ratio(0.0) > 3.3                       # second order with the load at t_{n+alpha_f}
    assert ratio(1.0 - E.genalpha(0.5)[1]) < 2.5  # the load at t_{n+1}: first order
