"""Pin of the oracle's adjoint gradient against central finite differences of
the whole forward integration (two generalized-alpha steps, Newton to 1e-13).
"""
import numpy as np
import pytest

import synth
from oracle import adjoint as AD


def _case(name):
    if name == "cube":
        mesh, mat, ti = synth.cube_case(2, nu=0.45, n_steps=2)
        sel = np.isclose(mesh.X[:, 2], 1.0)
        params = (0, 1)
    elif name == "tube":
        mesh, mat, ti = synth.tube_case(1, 8, 2, dt=0.05, n_steps=20)
        r = np.hypot(mesh.X[:, 0], mesh.X[:, 1])
        sel = np.isclose(r, 1.2)
        params = (0, 2, 3, 4)
    else:   # the eighth-strip: in-plane fibres at +-phi, dispersion, load ramped over 0.1 ms
        mesh, mat, ti = synth.strip_case(dims=(5, 3, 2), dt=1e-5, t_ramp=1e-4)
        sel = np.isclose(mesh.X[:, 0], 5e-3, rtol=0.0, atol=1e-12)
        params = (0, 2, 3, 4)
    return mesh, mat, ti, sel, params


def _J(mesh, mat, ti, theta, sel, target, n_steps):
    m2, mat2 = AD.with_params(mesh, mat, theta)
    states = AD.forward(m2, mat2, ti, n_steps)
    return AD.objective(states[-1]["u"], sel, target)[0]


@pytest.mark.parametrize("name", ["cube", "tube", "strip"])
def test_adjoint_gradient_matches_central_differences(name):
    mesh, mat, ti, sel, params = _case(name)
    n_steps = 2
    theta = AD.theta_of(mesh, mat)
    states = AD.forward(mesh, mat, ti, n_steps)
    u = states[-1]["u"]
    target = u[sel] * 0.9 + 1e-4 * np.random.default_rng(3).standard_normal(u[sel].shape)
    J, dJ = AD.objective(u, sel, target)
    grad = AD.adjoint_gradient(mesh, mat, ti, theta, states, dJ, params)
    for k in params:
        h = 1e-6 * max(abs(theta[k]), 1e-3)
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (_J(mesh, mat, ti, tp, sel, target, n_steps) - _J(mesh, mat, ti, tm, sel, target, n_steps)) / (2 * h)
        assert grad[k] == pytest.approx(fd, rel=1e-5, abs=1e-12 * abs(J) / max(abs(theta[k]), 1e-3)), AD.PARAMS[k]
