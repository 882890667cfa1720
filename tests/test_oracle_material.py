"""Pins for the oracle's constitutive relations (section 2; block-compression
and tensile-test energies in the numerical-results section).

The checks differentiate the paper's Gibbs energies numerically (complex
step / central differences) and compare with the oracle's closed forms, and
rebuild sigma_dev from its definition J^-1 F~ (P : S~) F~^T.
"""
import numpy as np
import pytest

import synth
from oracle import material as M

H_CS = 1e-30


def paper_gvol(p, kappa, rho0):
    # G_vol of the block-compression example, as printed in the paper
    s = np.sqrt(p ** 2 + kappa ** 2)
    return (p * s - p ** 2) / (2 * kappa * rho0) - kappa / (2 * rho0) * np.log((s - p) / kappa)


def paper_rho0_giso(Ct, mu, k1=0.0, k2=1.0, Hs=None):
    # rho0 * G_iso(C~): neo-Hookean matrix + fibre families (tensile-test example)
    W = mu / 2 * (np.trace(Ct) - 3)
    if Hs is not None:
        for H in Hs:
            E = np.sum(H * Ct) - 1
            W = W + k1 / (2 * k2) * (np.exp(k2 * E ** 2) - 1)
    return W


def cs_deriv(f, x):
    return np.imag(f(x + 1j * H_CS)) / H_CS


@pytest.mark.parametrize("kappa", [1e6, 5e7, 2.3e3])
def test_rho_beta_from_gibbs_energy(kappa):
    mat = synth.Material(kind=M.NH_COMP, rho0=1000.0, mu=1e5, kappa=kappa)
    for p in (-0.3 * kappa, -1e3, 0.0, 7e2, 0.45 * kappa):
        dG = cs_deriv(lambda q: paper_gvol(q, kappa, 1000.0), p)
        rho_num = 1.0 / dG
        # beta = -G'' / G' with G'' by central differences of the complex-step G'
        h = 1e-4 * max(abs(p), kappa)
        d2G = (cs_deriv(lambda q: paper_gvol(q, kappa, 1000.0), p + h)
               - cs_deriv(lambda q: paper_gvol(q, kappa, 1000.0), p - h)) / (2 * h)
        beta_num = -d2G / dG
        rho, beta, rho_p, beta_p = M.rho_beta(np.array(p), mat)
        assert rho == pytest.approx(rho_num, rel=1e-12, abs=0.0)
        assert beta == pytest.approx(beta_num, rel=1e-6, abs=0.0)
        # rho_p = d rho / dp, beta_p = d beta / dp (complex step of the closed forms'
        # definitions through the energy): rho_p = rho * beta by definition of beta
        drho = (1.0 / cs_deriv(lambda q: paper_gvol(q, kappa, 1000.0), p + h)
                - 1.0 / cs_deriv(lambda q: paper_gvol(q, kappa, 1000.0), p - h)) / (2 * h)
        assert rho_p == pytest.approx(drho, rel=1e-6, abs=0.0)
        b_hi = -1.0 / np.sqrt((p + h) ** 2 + kappa ** 2)
        b_lo = -1.0 / np.sqrt((p - h) ** 2 + kappa ** 2)
        assert beta_p == pytest.approx(-(b_hi - b_lo) / (2 * h), rel=1e-5, abs=1e-30)


def test_rest_and_incompressible_limits():
    mat = synth.Material(kind=M.NH_COMP, rho0=1000.0, mu=1e5, kappa=1e6)
    rho, beta, _, _ = M.rho_beta(np.array(0.0), mat)
    assert rho == pytest.approx(1000.0, rel=1e-15, abs=0.0)
    assert beta == pytest.approx(1e-6, rel=1e-15, abs=0.0)
    inc = synth.Material(kind=M.NH_INCOMP, rho0=1000.0, mu=1e5, kappa=np.inf)
    rho, beta, rp, bp = M.rho_beta(np.array([3e4, -2e4]), inc)
    assert np.all(rho == 1000.0) and np.all(beta == 0.0) and np.all(rp == 0) and np.all(bp == 0)
    big = synth.Material(kind=M.NH_COMP, rho0=1000.0, mu=1e5, kappa=1e14)
    rho, beta, _, _ = M.rho_beta(np.array(3e4), big)
    assert rho == pytest.approx(1000.0, rel=1e-9, abs=0.0) and beta < 1e-13


def _random_F(rng, amp=0.2):
    F = np.eye(3) + amp * rng.uniform(-1, 1, (3, 3))
    assert np.linalg.det(F) > 0
    return F


def _fibre_H(rng, kd):
    a = rng.standard_normal((2, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    return np.array([kd * np.eye(3) + (1 - 3 * kd) * np.outer(x, x) for x in a]), a


@pytest.mark.parametrize("kind", [M.NH_COMP, M.HGO_INCOMP])
def test_piola_is_energy_gradient(kind):
    rng = np.random.default_rng(3)
    mat = synth.Material(kind=kind, rho0=1000.0, mu=3e4, kappa=1e6, k1=2.36e5, k2=0.84, kd=0.1)
    for _ in range(5):
        F = _random_F(rng)
        Hs, _ = _fibre_H(rng, mat.kd)
        Hs_use = Hs if kind == M.HGO_INCOMP else None

        def W(Fc):
            J = np.linalg.det(Fc)
            Ct = J ** (-2 / 3) * Fc.T @ Fc
            return paper_rho0_giso(Ct, mat.mu, mat.k1, mat.k2, Hs_use)

        dW = np.zeros((3, 3))
        for i in range(3):
            for I in range(3):
                E = np.zeros((3, 3), dtype=complex)
                E[i, I] = 1j * H_CS
                dW[i, I] = np.imag(W(F + E)) / H_CS
        P = M.piola_iso(F[None], mat, Hs[None] if Hs_use is not None else None)[0]
        np.testing.assert_allclose(P, dW, rtol=1e-12, atol=1e-10 * np.abs(dW).max())


@pytest.mark.parametrize("kind", [M.NH_COMP, M.HGO_INCOMP])
def test_sigma_dev_from_projection_definition(kind):
    """sigma_dev = J^-1 F~ (P : S~) F~^T with S~ = 2 d(rho0 G_iso)/dC~ and the
    deviatoric projector P = I - 1/3 C~^-1 (x) C~; P~ = J sigma_dev F^-T."""
    rng = np.random.default_rng(11)
    mat = synth.Material(kind=kind, rho0=1000.0, mu=3e4, kappa=1e6, k1=2.36e5, k2=0.84, kd=0.2)
    for _ in range(5):
        F = _random_F(rng)
        Hs, _ = _fibre_H(rng, mat.kd)
        Hs_use = Hs if kind == M.HGO_INCOMP else None
        J = np.linalg.det(F)
        Ct = J ** (-2 / 3) * F.T @ F
        St = np.zeros((3, 3))
        for I in range(3):
            for K in range(3):
                E = np.zeros((3, 3), dtype=complex)
                E[I, K] = 1j * H_CS
                St[I, K] = 2 * np.imag(paper_rho0_giso(Ct + E, mat.mu, mat.k1, mat.k2, Hs_use)) / H_CS
        PS = St - np.sum(Ct * St) / 3 * np.linalg.inv(Ct)
        Ft = J ** (-1 / 3) * F
        sig = Ft @ PS @ Ft.T / J
        assert abs(np.trace(sig)) < 1e-9 * np.abs(sig).max()
        P_def = J * sig @ np.linalg.inv(F).T
        P = M.piola_iso(F[None], mat, Hs[None] if Hs_use is not None else None)[0]
        np.testing.assert_allclose(P, P_def, rtol=1e-10, atol=1e-10 * np.abs(P).max())


def test_neo_hookean_textbook_cauchy():
    """neo-Hookean isochoric Cauchy stress is mu J^(-5/3) dev(F F^T)."""
    rng = np.random.default_rng(5)
    mat = synth.Material(kind=M.NH_COMP, mu=7.0e4)
    F = _random_F(rng)
    J = np.linalg.det(F)
    b = F @ F.T
    sig = mat.mu * J ** (-5 / 3) * (b - np.trace(b) / 3 * np.eye(3))
    P = M.piola_iso(F[None], mat)[0]
    np.testing.assert_allclose(P @ F.T / J, sig, rtol=1e-12, atol=1e-9)


def test_kind_constants_match_inputs():
    assert (M.NH_COMP, M.NH_INCOMP, M.HGO_INCOMP) == (synth.NH_COMP, synth.NH_INCOMP, synth.HGO_INCOMP)


def test_wave_speed_and_kappa_of_nu():
    # the block benchmark's mu, kappa correspond to nu = 0.4999 (to the printed digits)
    mu, kappa = 80.194, 400889.806
    assert (3 * kappa - 2 * mu) / (2 * (3 * kappa + mu)) == pytest.approx(0.4999, abs=5e-8)
    mat = synth.material_from_nu(mu, (3 * kappa - 2 * mu) / (2 * (3 * kappa + mu)))
    assert mat.kappa == pytest.approx(kappa, rel=1e-12, abs=0.0)
    m2 = synth.material_from_nu(1e5, 0.45)
    assert M.wave_speed(m2) == pytest.approx(np.sqrt((m2.kappa + 4e5 / 3) / 1000.0), rel=1e-12, abs=0.0)
    inc = synth.material_from_nu(1e5, 0.5)
    assert inc.kind == M.NH_INCOMP and M.wave_speed(inc) == pytest.approx(10.0, rel=1e-12, abs=0.0)
