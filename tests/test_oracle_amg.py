"""Pins for the oracle's aggregation multigrid (oracle/amg.py), against what the
mathematics fixes rather than against itself:

* SplitMix64 reproduces the generator's published first outputs;
* the aggregation of a path graph equals the hand-worked partition, and on a
  mesh graph every node lies in exactly one connected aggregate, phase-1
  aggregates being closed neighbourhoods;
* translations, rotations and the dilation lie in the kernel of the
  linearised isochoric stiffness of the P1 mesh (exactly: they are linear
  fields), and the special conformal fields nearly so, unlike other quadratics;
* the tentative prolongator is orthonormal and reproduces the near-null space
  (B = Q R);
* with singleton aggregates the coarse space is the whole space, so a two-level
  cycle with an exact coarse solve is the exact inverse;
* the Chebyshev smoother applies the textbook Chebyshev polynomial;
* the power estimate bounds the top eigenvalue from below within a few %;
* the V-cycle is a symmetric positive definite operator, and CG with it
  reaches the sparse LU solution of the A-block.
"""
import os

import numpy as np
import numpy.polynomial.chebyshev as npcheb
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import amg as AMG
from oracle import assemble as AS
from oracle import element as E

HERE = os.path.dirname(os.path.abspath(__file__))


def _scaled_A(mesh, mat, dt, sym=True):
    disc = AS.Discretization(mesh, mat)
    am, af, gm = E.genalpha(0.5)
    n = mesh.n_nodes
    st = {k: np.zeros((n, 3)) for k in ("u", "v", "du", "dv")}
    st["p"], st["dp"] = np.zeros(n), np.zeros(n)
    K = disc.tangent(st, (am, af, gm, dt))
    Kd, _ = AS.apply_dirichlet(K, np.zeros(K.shape[0]), disc.dof_dir)
    W = AS.scaling(Kd)
    Ks = Kd.multiply(W[:, None]).multiply(W[None, :]).tocsr()
    A, _, _, _, iv, _ = AS.split_blocks(Ks)
    if sym:
        A = ((A + A.T) * 0.5).tocsr()
    return A, W[iv].reshape(n, 3)


def test_splitmix64_published_outputs():
    want = [int(line, 16) for line in open(os.path.join(HERE, "golden", "splitmix64_seed0.txt"))
            if line.strip() and not line.startswith("#")]
    assert [AMG.splitmix64_raw(0, i) for i in range(3)] == want
    v = AMG.splitmix64(5, 1000)
    assert v.min() >= -1.0 and v.max() < 1.0 and abs(v.mean()) < 0.1


def test_aggregation_of_a_path_graph():
    # path 0-1-2-3-4-5-6 with self loops: phase 1 takes {0,1} and {2,3,4} ... by hand:
    # node 0: {0,1} free -> aggregate 0; node 2: neighbour 1 taken; node 3: {2,3,4} -> aggregate 1;
    # node 5: neighbour 4 taken; node 6: {5,6} -> aggregate 2; nothing is left for phases 2, 3
    n = 7
    r = np.concatenate([np.arange(n), np.arange(n - 1), np.arange(1, n)])
    c = np.concatenate([np.arange(n), np.arange(1, n), np.arange(n - 1)])
    G = sp.csr_matrix((np.ones(r.size), (r, c)), shape=(n, n))
    agg, na = AMG.aggregate(G.indptr, G.indices)
    assert na == 3 and agg.tolist() == [0, 0, 1, 1, 1, 2, 2]
    # an 8-node path leaves node 7 for phase 2: it joins its neighbour 6's aggregate
    n = 8
    r = np.concatenate([np.arange(n), np.arange(n - 1), np.arange(1, n)])
    c = np.concatenate([np.arange(n), np.arange(1, n), np.arange(n - 1)])
    G = sp.csr_matrix((np.ones(r.size), (r, c)), shape=(n, n))
    agg, na = AMG.aggregate(G.indptr, G.indices)
    assert na == 3 and agg.tolist() == [0, 0, 1, 1, 1, 2, 2, 2]


@pytest.mark.parametrize("case", ["cube", "tube"])
def test_aggregates_partition_the_mesh_graph(case):
    mesh = synth.cube_case(5)[0] if case == "cube" else synth.tube_case(2, 12, 6)[0]
    G = AMG.mesh_graph(mesh.tets, mesh.n_nodes)
    agg, na = AMG.aggregate(G.indptr, G.indices)
    assert agg.min() == 0 and agg.max() == na - 1
    mem = AMG.members(agg, na)
    assert sum(len(m) for m in mem) == mesh.n_nodes
    for a, nodes in enumerate(mem):
        sub = G[nodes][:, nodes]
        ncomp, _ = sp.csgraph.connected_components(sub, directed=False)
        assert ncomp == 1, a
    # a phase-1 aggregate: some member's whole neighbourhood lies inside it
    closed = sum(any(set(G.indices[G.indptr[i]:G.indptr[i + 1]]) <= set(nodes) for i in nodes) for nodes in mem)
    assert closed >= na * 0.5


def _iso_stiffness(mesh, mat):
    """Linearised isochoric stiffness at rest: the velocity block of the
    tangent is alpha_m rho0 M + (alpha_f gamma dt)^2 / alpha_m K, so two time
    steps separate K."""
    disc = AS.Discretization(mesh, mat)
    am, af, gm = E.genalpha(0.5)
    n = mesh.n_nodes
    st = {k: np.zeros((n, 3)) for k in ("u", "v", "du", "dv")}
    st["p"], st["dp"] = np.zeros(n), np.zeros(n)
    A = []
    for dt in (1e-3, 2e-3):
        K = disc.tangent(st, (am, af, gm, dt))
        A.append(AS.split_blocks(K)[0])
    c = (af * gm) ** 2 / am * (2e-3 ** 2 - 1e-3 ** 2)
    return ((A[1] - A[0]) / c).tocsr()


@pytest.mark.parametrize("kind", ["nh", "hgo"])
def test_conformal_modes_span_the_isochoric_kernel(kind):
    if kind == "nh":
        mesh, _, _ = synth.cube_case(4)
        mat = synth.material_from_nu(1e5, 0.5)
    else:
        mesh, mat, _ = synth.tube_case(2, 12, 6)
    K = _iso_stiffness(mesh, mat)
    Y = mesh.X - mesh.X.mean(axis=0)
    Y /= np.abs(Y).max()
    B = AMG.conformal_modes(Y).reshape(3 * mesh.n_nodes, AMG.NMODES)
    kn = spla.norm(K)
    rel = [np.linalg.norm(K @ B[:, k]) / (kn * np.linalg.norm(B[:, k])) for k in range(AMG.NMODES)]
    # linear fields: translations, rotations, dilation are in the discrete kernel
    assert max(rel[:7]) < 1e-12, rel
    # quadratic special conformal fields: nearly in the kernel, far closer than
    # a quadratic that is not conformal (the same field with the opposite sign of |y|^2)
    s2 = np.sum(Y * Y, axis=1)
    for a in range(3):
        other = 2.0 * Y[:, a:a + 1] * Y
        other[:, a] += s2
        ro = np.linalg.norm(K @ other.ravel()) / (kn * np.linalg.norm(other))
        assert rel[7 + a] < 0.5 * ro, (a, rel[7 + a], ro)


def test_tentative_prolongator_is_orthonormal_and_reproduces_the_modes():
    mesh, _, _ = synth.tube_case(2, 12, 6)
    G = AMG.mesh_graph(mesh.tets, mesh.n_nodes)
    agg, na = AMG.aggregate(G.indptr, G.indices)
    mem = AMG.members(agg, na)
    dv = mesh.dir_mask[:, 0:3].astype(bool)
    B = AMG.fine_modes(mesh.X, mem, dv)
    Q, R, dropped = AMG.tentative(mem, B, 3)
    QtQ = (Q.T @ Q).toarray()
    keep = ~dropped
    np.testing.assert_allclose(QtQ[np.ix_(keep, keep)], np.eye(keep.sum()), atol=1e-12)
    assert np.abs(QtQ[dropped]).max(initial=0.0) == 0.0
    # B restricted to each aggregate equals Q R
    for a, nodes in enumerate(mem):
        dofs = (nodes[:, None] * 3 + np.arange(3)).ravel()
        Qa = Q[dofs][:, a * 10:(a + 1) * 10].toarray()
        np.testing.assert_allclose(Qa @ R[a * 10:(a + 1) * 10], B[dofs], atol=1e-12)
    # aggregates reach past the clamped end into the interior: few coarse dofs are dropped
    assert (~dropped).sum() > 0.7 * dropped.size


def test_two_level_with_singleton_aggregates_is_exact():
    mesh, mat, _ = synth.tube_case(1, 8, 4)
    A, W = _scaled_A(mesh, mat, 0.05)
    n = mesh.n_nodes
    eye = sp.identity(n, format="csr")           # no edges: every aggregate is one node
    lev = AMG.build(A, W, mesh.X, mesh.dir_mask[:, 0:3].astype(bool), max_levels=2, min_coarse=0, graph=eye)
    assert len(lev) == 2 and lev[0].P.shape[1] == 10 * n
    b = np.random.default_rng(3).standard_normal(3 * n)
    b[mesh.dir_mask[:, 0:3].astype(bool).ravel()] = 0.0   # the solves' Dirichlet rows carry zero
    x = AMG.vcycle(lev, b, coarse_solve=lambda Ac, r: spla.spsolve(Ac.tocsc(), r))
    xe = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - xe) <= 1e-10 * np.linalg.norm(xe)


@pytest.mark.parametrize("degree", [1, 2, 3, 5])
def test_chebyshev_smoother_is_the_chebyshev_polynomial(degree):
    lam = np.linspace(0.01, 2.0, 60)
    L = AMG.Level()
    L.A = sp.diags(lam).tocsr()
    L.Dinv = sp.identity(lam.size, format="csr")
    L.lmax = 2.0
    e = np.random.default_rng(4).standard_normal(lam.size)
    x = AMG.chebyshev(L, L.A @ e, None, degree)
    lmin = L.lmax / AMG.CHEB_RATIO
    theta, delta = 0.5 * (L.lmax + lmin), 0.5 * (L.lmax - lmin)
    Tk = np.zeros(degree + 1)
    Tk[degree] = 1.0
    p = npcheb.chebval((theta - lam) / delta, Tk) / npcheb.chebval(theta / delta, Tk)
    np.testing.assert_allclose(e - x, p * e, atol=1e-12 * np.abs(e).max())


def test_power_estimate_bounds_the_top_eigenvalue():
    lam = np.concatenate([np.linspace(0.1, 1.0, 500), [1.3]])
    A = sp.diags(lam).tocsr()
    est = AMG.power_lmax(A, sp.identity(lam.size, format="csr"), seed=3) / AMG.LMAX_SAFETY
    assert 0.95 * 1.3 <= est <= 1.3


@pytest.mark.parametrize("mid_degree", [0, 3])
def test_vcycle_is_symmetric_positive_definite(mid_degree):
    mesh, mat, _ = synth.tube_case(2, 16, 8)
    A, W = _scaled_A(mesh, mat, 0.05)
    lev = AMG.build(A, W, mesh.X, mesh.dir_mask[:, 0:3].astype(bool), max_levels=3, min_coarse=10,
                    graph=AMG.mesh_graph(mesh.tets, mesh.n_nodes))
    assert len(lev) >= 2
    rng = np.random.default_rng(8)
    a, b = rng.standard_normal((2, A.shape[0]))
    Va, Vb = AMG.vcycle(lev, a, mid_degree=mid_degree), AMG.vcycle(lev, b, mid_degree=mid_degree)
    assert abs(Va @ b - a @ Vb) <= 1e-12 * np.linalg.norm(Va) * np.linalg.norm(b)
    assert Va @ a > 0.0 and Vb @ b > 0.0


def test_middle_level_smoothing_tends_to_the_two_grid_cycle():
    """With an exact solve on the coarsest of three levels, raising the middle level's degree
    makes its sub-cycle an ever better solve with that level's operator: the three-level cycle
    tends to the two-level one whose second level is solved exactly, while the finest level keeps
    its own degree."""
    mesh, mat, _ = synth.tube_case(2, 16, 8)
    A, W = _scaled_A(mesh, mat, 0.05)
    lev = AMG.build(A, W, mesh.X, mesh.dir_mask[:, 0:3].astype(bool), max_levels=3, min_coarse=10,
                    graph=AMG.mesh_graph(mesh.tets, mesh.n_nodes))
    assert len(lev) == 3
    exact = lambda Ac, r: spla.spsolve(Ac.tocsc(), r)
    b = np.random.default_rng(9).standard_normal(A.shape[0])
    b[mesh.dir_mask[:, 0:3].astype(bool).ravel()] = 0.0
    two = AMG.vcycle(lev[:2], b, degree=2, coarse_solve=exact)
    gap = [np.linalg.norm(AMG.vcycle(lev, b, degree=2, coarse_solve=exact, mid_degree=k) - two)
           / np.linalg.norm(two) for k in (1, 2, 4, 8, 16)]
    assert all(g1 < g0 for g0, g1 in zip(gap, gap[1:])), gap
    assert gap[-1] < 1e-3 * gap[0], gap
    # mid_degree equal to degree is the plain cycle
    np.testing.assert_array_equal(AMG.vcycle(lev, b, degree=2, mid_degree=2), AMG.vcycle(lev, b, degree=2))


def test_amg_cg_reaches_the_lu_solution_faster_than_block_jacobi():
    mesh, mat, _ = synth.tube_case(2, 24, 12)
    A, W = _scaled_A(mesh, mat, 0.05)
    lev = AMG.build(A, W, mesh.X, mesh.dir_mask[:, 0:3].astype(bool),
                    graph=AMG.mesh_graph(mesh.tets, mesh.n_nodes))
    b = np.random.default_rng(9).standard_normal(A.shape[0])
    b[mesh.dir_mask[:, 0:3].astype(bool).ravel()] = 0.0
    x, its = AMG.pcg(A, b, lambda r: AMG.vcycle(lev, r), 1e-10)
    xe = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - xe) <= 1e-8 * np.linalg.norm(xe)
    Dinv = AMG.block_diag_inv(A, 3)
    _, its_bj = AMG.pcg(A, b, lambda r: Dinv @ r, 1e-10)
    print(f"[amg] levels={[L.A.shape[0] for L in lev]} cg its: amg {its}, block-Jacobi {its_bj}")
    assert its < 0.5 * its_bj


def test_coarse_operator_does_not_depend_on_the_scaling():
    """x = W x*: the prolongator of the scaled system is W^-1 Q, so the coarse
    operator of W A W equals that of A built with W = 1 (section 4.1's scaling
    leaves the coarse levels unchanged)."""
    mesh, mat, _ = synth.tube_case(2, 12, 6)
    As, W = _scaled_A(mesh, mat, 0.05)
    Au = (sp.diags(1.0 / W.ravel()) @ As @ sp.diags(1.0 / W.ravel())).tocsr()
    dv = mesh.dir_mask[:, 0:3].astype(bool)
    G = AMG.mesh_graph(mesh.tets, mesh.n_nodes)
    ls = AMG.build(As, W, mesh.X, dv, max_levels=2, min_coarse=0, graph=G)
    lu = AMG.build(Au, np.ones_like(W), mesh.X, dv, max_levels=2, min_coarse=0, graph=G)
    d = (ls[1].A - lu[1].A).tocsr()
    assert abs(d).max() <= 1e-12 * abs(lu[1].A).max()
    assert np.max(np.abs(W - 1.0)) > 0.5          # the scaling is far from the identity
