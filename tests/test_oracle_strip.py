"""The tensile-strip workload of section 5.2 and the fibre dispersion it uses.

* mesh data: the eighth-strip fills [0, 5] x [0, 1.5] x [0, 0.25] mm with
  positively oriented tets, its symmetry-plane nodes lie on their planes and
  carry the symmetry conditions, the loading face is held to move along x;
* the oracle's nodal load of the dead traction sums to a quarter of the
  tensile force (the eighth's share of the specimen's cross-section);
* the structure tensors H_i = k_d I + (1 - 3 k_d) a_i (x) a_i: unit trace,
  a_i an eigenvector with eigenvalue 1 - 2 k_d, k_d = 0 gives a_i (x) a_i and
  k_d = 1/3 gives I/3 whatever the fibre;
* with k_d = 1/3 the fibre energy depends on tr C~ only, so the oracle's iso
  Piola stress must equal the closed form of an isotropic I1 material,
  P~ = (mu + 2s) J^(-2/3) (F - tr C / 3 F^-T) with
  s = (2/3) k1 E e^(k2 E^2), E = J^(-2/3) tr C / 3 - 1, for any fibres;
* the oracle's Newton iteration on a small strip at the paper's dt = 0.1
  converges quadratically.
"""
import numpy as np
import pytest

import synth
from oracle import assemble as AS
from oracle import material as M
from oracle import newton as NW


def _strip(dims=(10, 4, 3), **kw):
    return synth.strip_case(dims=dims, **kw)


def test_strip_dims_follow_the_mesh_ladder():
    assert synth.strip_dims(200) == (200, 60, 10)
    assert synth.strip_dims(400) == (400, 120, 20)
    assert synth.strip_dims(600) == (600, 180, 30)


def test_strip_geometry_and_boundary_conditions():
    mesh, mat, ti = _strip()
    X, t = mesh.X, mesh.tets
    vol = np.linalg.det(X[t[:, 1:]] - X[t[:, [0]]]) / 6.0
    assert vol.min() > 0.0
    assert vol.sum() == pytest.approx(5e-3 * 1.5e-3 * 0.25e-3, rel=1e-12)
    lo, hi = X.min(axis=0), X.max(axis=0)
    np.testing.assert_allclose(lo, 0.0, atol=0.0)
    np.testing.assert_allclose(hi, [5e-3, 1.5e-3, 0.25e-3], rtol=1e-15)
    on = [np.isclose(X[:, c], 0.0, atol=0.0) for c in range(3)]
    far = np.isclose(X[:, 0], 5e-3, rtol=0.0, atol=1e-18)
    # symmetry planes: exactly on the plane, normal component fixed, nothing else
    for c in range(3):
        assert mesh.dir_mask[on[c], c].all()
    expect = np.stack([on[0], on[1] | far, on[2] | far], axis=1)
    np.testing.assert_array_equal(mesh.dir_mask[:, 0:3].astype(bool), expect)
    assert not mesh.dir_mask[:, 3].any()
    assert not mesh.dir_vel.any()
    # loaded faces: on x = 5 mm, covering the eighth's cross-section
    assert far[mesh.bfaces].all()
    a, b, c = (X[mesh.bfaces[:, k]] for k in range(3))
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    assert area.sum() == pytest.approx(1.5e-3 * 0.25e-3, rel=1e-12)
    assert mesh.n_nodes == 11 * 5 * 4 and mesh.n_tets == 6 * 10 * 4 * 3


def test_strip_fibres_are_in_plane_at_plus_minus_phi():
    mesh, _, _ = _strip(fibre_deg=40.02)
    f = mesh.fibre
    np.testing.assert_allclose(np.linalg.norm(f, axis=2), 1.0, rtol=1e-15)
    assert not f[:, :, 2].any()
    ang = np.degrees(np.arctan2(f[:, :, 1], f[:, :, 0]))
    np.testing.assert_allclose(ang[:, 0], 40.02, rtol=1e-13)
    np.testing.assert_allclose(ang[:, 1], -40.02, rtol=1e-13)
    fib, dfib = synth.fibre_field(mesh, np.deg2rad(40.02) + 1e-30j)
    np.testing.assert_allclose(np.imag(fib) / 1e-30, dfib, rtol=1e-14, atol=1e-15)


def test_strip_nodal_load_is_a_quarter_of_the_force():
    mesh, mat, _ = _strip()
    f = AS.Discretization(mesh, mat).nodal_traction(1.0)
    np.testing.assert_allclose(f.sum(axis=0), [-0.5, 0.0, 0.0], atol=1e-15)
    half = AS.Discretization(mesh, mat).nodal_traction(0.5)
    np.testing.assert_allclose(half, 0.5 * f, rtol=1e-15)


@pytest.mark.parametrize("kd", [0.0, 0.1, 0.226, 1.0 / 3.0])
def test_structure_tensor_properties(kd):
    rng = np.random.default_rng(5)
    a = rng.standard_normal((7, 2, 3))
    a /= np.linalg.norm(a, axis=2, keepdims=True)
    H = M.structure_tensors(a, kd)
    np.testing.assert_allclose(np.trace(H, axis1=2, axis2=3), 1.0, rtol=1e-14)
    np.testing.assert_allclose(np.einsum("mfij,mfj->mfi", H, a), (1 - 2 * kd) * a, atol=1e-15)
    np.testing.assert_allclose(H, np.swapaxes(H, 2, 3), atol=0.0)
    if kd == 0.0:
        np.testing.assert_allclose(H, a[..., :, None] * a[..., None, :], atol=0.0)
    if kd == 1.0 / 3.0:
        np.testing.assert_allclose(H, np.broadcast_to(np.eye(3) / 3.0, H.shape), atol=1e-16)


def test_isotropic_dispersion_gives_closed_form_i1_stress():
    mat = synth.Material(kind=M.HGO_INCOMP, rho0=1000.0, mu=7.64e3, kappa=np.inf,
                         k1=996.6e3, k2=524.6, kd=1.0 / 3.0)
    rng = np.random.default_rng(11)
    for _ in range(4):
        F = np.eye(3) + 0.05 * rng.standard_normal((3, 3))
        J = np.linalg.det(F)
        trC = np.trace(F.T @ F)
        E_ = J ** (-2.0 / 3.0) * trC / 3.0 - 1.0
        s = (2.0 / 3.0) * mat.k1 * E_ * np.exp(mat.k2 * E_ ** 2)
        P = (mat.mu + 2.0 * s) * J ** (-2.0 / 3.0) * (F - trC / 3.0 * np.linalg.inv(F).T)
        for _ in range(2):
            a = rng.standard_normal((1, 2, 3))
            a /= np.linalg.norm(a, axis=2, keepdims=True)
            Po = M.piola_iso(F[None], mat, M.structure_tensors(a, mat.kd))[0]
            np.testing.assert_allclose(Po, P, rtol=1e-11, atol=1e-11 * np.abs(P).max())


def test_oracle_newton_on_strip_converges_quadratically():
    mesh, mat, ti = _strip(dt=0.1)
    disc = AS.Discretization(mesh, mat)
    st = NW.rest_state(mesh)
    for s in range(2):
        st, info = NW.time_step(disc, ti, st, s * ti.dt, tol_R=1e-11)
        assert info["converged"]
        r = np.array(info["norms"]) / info["norms"][0]
        # contractions above the round-off floor (~1e-12 here) are quadratic:
        # r_{l+1} <= C r_l^2 once r_l is small
        small = [(r[l], r[l + 1]) for l in range(len(r) - 1) if r[l] < 1e-3 and r[l + 1] > 1e-10]
        assert small and all(b <= 1e3 * a * a for a, b in small), r
    assert st["u"][:, 0].max() > 0.0          # the strip stretches along the load
