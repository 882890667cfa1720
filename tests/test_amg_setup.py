"""The library's host-side multigrid set-up (vms_amg_create, no GPU needed)
against the oracle's hierarchy on the same meshes: aggregates and coarse
patterns bit for bit (integer work), dropped coarse dofs equal, tentative
prolongators and their coarse near-null spaces to rounding."""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import amg as AMG
from paper_1809_06350_amd import _lib as L
from paper_1809_06350_amd import vms as V

from test_abi import build_host


def _plan(mesh, opts):
    lib = L.load()
    h = build_host(mesh)
    X = np.ascontiguousarray(mesh.X, np.float64)
    dm = np.ascontiguousarray(mesh.dir_mask, np.uint8)
    obj = C.c_void_p()
    rc = lib.vms_amg_create(mesh.n_nodes, h["W"], h["row_len"].ctypes.data, h["col"].ctypes.data, X.ctypes.data,
                            dm.ctypes.data, C.byref(opts), C.byref(obj))
    assert rc == 0
    return lib, obj


def _level(lib, obj, level, n, bs, nnzb):
    ptrs = [C.c_void_p() for _ in range(5)]
    assert lib.vms_amg_level_arrays(obj, level, *(C.byref(p) for p in ptrs)) == 0
    out = {}
    if ptrs[0].value:
        out["agg"] = np.ctypeslib.as_array(C.cast(ptrs[0], C.POINTER(C.c_int32)), (n,)).copy()
        out["P"] = np.ctypeslib.as_array(C.cast(ptrs[1], C.POINTER(C.c_double)), (n * bs * 10,)).copy()
    if level > 0:
        out["ptr"] = np.ctypeslib.as_array(C.cast(ptrs[2], C.POINTER(C.c_int32)), (n + 1,)).copy()
        out["col"] = np.ctypeslib.as_array(C.cast(ptrs[3], C.POINTER(C.c_int32)), (nnzb,)).copy()
        out["dropped"] = np.ctypeslib.as_array(C.cast(ptrs[4], C.POINTER(C.c_uint8)), (n * 10,)).copy()
    return out


def _oracle_hierarchy(mesh, max_levels, min_coarse):
    """The oracle's aggregates, unscaled prolongators Q, dropped masks and coarse graphs, level by level."""
    G = AMG.mesh_graph(mesh.tets, mesh.n_nodes)
    dv = mesh.dir_mask[:, 0:3].astype(bool)
    out, B, blk = [], None, 3
    for lev in range(max_levels):
        nn = G.shape[0]
        if lev == max_levels - 1 or nn <= min_coarse:
            out.append({"n": nn})
            break
        agg, na = AMG.aggregate(G.indptr, G.indices)
        mem = AMG.members(agg, na)
        if lev == 0:
            B = AMG.fine_modes(mesh.X, mem, dv)
        Q, R, dropped = AMG.tentative(mem, B, blk)
        out.append({"n": nn, "agg": agg, "Q": Q, "dropped_next": dropped})
        Pa = sp.csr_matrix((np.ones(nn), (np.arange(nn), agg)), shape=(nn, na))
        G = (Pa.T @ G @ Pa).tocsr()
        G.sort_indices()
        G.data[:] = 1.0
        out[-1]["G_next"] = G
        B, blk = R, 10
    return out


@pytest.mark.parametrize("case", ["cube", "tube", "strip"])
def test_host_hierarchy_matches_oracle(case):
    if case == "cube":
        mesh = synth.cube_case(6)[0]
    elif case == "tube":
        mesh = synth.tube_case(2, 16, 10)[0]
    else:
        mesh = synth.strip_case(dims=(12, 6, 3))[0]
    opts = V.amg_opts(max_levels=4, min_coarse=8)
    lib, obj = _plan(mesh, opts)
    try:
        info = L.AmgInfo()
        assert lib.vms_amg_get_info(obj, C.byref(info)) == 0
        ora = _oracle_hierarchy(mesh, 4, 8)
        assert info.n_levels == len(ora) >= 2
        for lev in range(info.n_levels):
            n, bs = info.n[lev], info.bs[lev]
            assert n == ora[lev]["n"]
            got = _level(lib, obj, lev, n, bs, info.nnzb[lev])
            if "agg" in ora[lev]:
                assert np.array_equal(got["agg"], ora[lev]["agg"]), lev
                Q = ora[lev]["Q"].toarray().reshape(n, bs, -1, 10)
                agg = ora[lev]["agg"]
                Pq = Q[np.arange(n), :, agg, :]        # each node's block in its own aggregate's columns
                np.testing.assert_allclose(got["P"].reshape(n, bs, 10), Pq, rtol=0, atol=1e-12)
                Gn = ora[lev]["G_next"]
                nxt = _level(lib, obj, lev + 1, info.n[lev + 1], info.bs[lev + 1], info.nnzb[lev + 1])
                assert np.array_equal(nxt["ptr"], Gn.indptr) and np.array_equal(nxt["col"], Gn.indices)
                assert np.array_equal(nxt["dropped"].astype(bool), ora[lev]["dropped_next"])
    finally:
        lib.vms_amg_destroy(obj)


def test_amg_create_rejects_bad_input():
    lib = L.load()
    mesh = synth.cube_case(2)[0]
    h = build_host(mesh)
    X = np.ascontiguousarray(mesh.X, np.float64)
    dm = np.ascontiguousarray(mesh.dir_mask, np.uint8)
    obj = C.c_void_p()
    for opts in (V.amg_opts(max_levels=1), V.amg_opts(max_levels=9), V.amg_opts(degree=0),
                 V.amg_opts(coarse_degree=65), V.amg_opts(min_coarse=-1),
                 V.amg_opts(mid_degree=-1), V.amg_opts(mid_degree=17)):
        assert lib.vms_amg_create(mesh.n_nodes, h["W"], h["row_len"].ctypes.data, h["col"].ctypes.data,
                                  X.ctypes.data, dm.ctypes.data, C.byref(opts), C.byref(obj)) == -1
    bad = h["col"].copy()
    bad[1] = mesh.n_nodes + 5
    assert lib.vms_amg_create(mesh.n_nodes, h["W"], h["row_len"].ctypes.data, bad.ctypes.data, X.ctypes.data,
                              dm.ctypes.data, C.byref(V.amg_opts()), C.byref(obj)) == -1
