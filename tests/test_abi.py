"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/vms.h declares, and its integer setup (block
pattern, transpose map, element->block map, colouring, node->face lists) is
exact against independent constructions."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from paper_1809_06350_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "vms.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(vms_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 16
    for name in names:
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, f"{name} has no ctypes signature"
    assert set(L.SIGNATURES) == set(names)


def build_host(mesh):
    lib = L.load()
    n, m, f = mesh.n_nodes, mesh.n_tets, mesh.bfaces.shape[0]
    tets = np.ascontiguousarray(mesh.tets, np.int32)
    bf = np.ascontiguousarray(mesh.bfaces, np.int32)
    nnzb, ncb = C.c_int64(), C.c_int32()
    assert lib.vms_setup_sizes(n, m, tets.ctypes.data, C.byref(nnzb), C.byref(ncb)) == 0
    nz = nnzb.value
    h = {"row_ptr": np.zeros(n + 1, np.int32), "col": np.zeros(nz, np.int32), "tpos": np.zeros(nz, np.int32),
         "diag_pos": np.zeros(n, np.int32), "elem_blk": np.zeros(16 * m, np.int32),
         "colour_ptr": np.zeros(ncb.value + 1, np.int32), "elem_by_colour": np.zeros(m, np.int32),
         "nf_ptr": np.zeros(n + 1, np.int32), "nf_face": np.zeros(max(3 * f, 1), np.int32)}
    ncol = C.c_int32()
    rc = lib.vms_setup_build(n, m, tets.ctypes.data, f, bf.ctypes.data,
                             *(h[k].ctypes.data for k in ("row_ptr", "col", "tpos", "diag_pos", "elem_blk",
                                                          "colour_ptr", "elem_by_colour")),
                             C.byref(ncol), h["nf_ptr"].ctypes.data, h["nf_face"].ctypes.data)
    assert rc == 0
    h["n_colours"] = ncol.value
    h["colour_ptr"] = h["colour_ptr"][: ncol.value + 1]
    return h


@pytest.mark.parametrize("N", [1, 3, 4])
def test_pattern_matches_element_connectivity(N):
    mesh = synth.cube_mesh(N)
    h = build_host(mesh)
    n = mesh.n_nodes
    # independent construction: node pairs sharing a tet
    t = mesh.tets
    r = np.repeat(t, 4, axis=1).ravel()
    c = np.tile(t, (1, 4)).ravel()
    G = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(n, n)).tocsr()
    G.sum_duplicates()
    G.sort_indices()
    np.testing.assert_array_equal(h["row_ptr"], G.indptr)
    np.testing.assert_array_equal(h["col"], G.indices)
    rows = np.repeat(np.arange(n), np.diff(G.indptr))
    col = h["col"]
    # transpose map and diagonal positions
    np.testing.assert_array_equal(rows[h["tpos"]], col)
    np.testing.assert_array_equal(col[h["tpos"]], rows)
    np.testing.assert_array_equal(col[h["diag_pos"]], np.arange(n))
    np.testing.assert_array_equal(rows[h["diag_pos"]], np.arange(n))
    # element -> block map
    eb = h["elem_blk"].reshape(-1, 4, 4)
    np.testing.assert_array_equal(rows[eb], np.repeat(t[:, :, None], 4, axis=2))
    np.testing.assert_array_equal(col[eb], np.repeat(t[:, None, :], 4, axis=1))


@pytest.mark.parametrize("N", [2, 4, 6])
def test_colouring_is_conflict_free_and_complete(N):
    mesh = synth.cube_mesh(N)
    h = build_host(mesh)
    cp, ebc = h["colour_ptr"], h["elem_by_colour"]
    assert cp[-1] == mesh.n_tets
    assert np.array_equal(np.sort(ebc), np.arange(mesh.n_tets))
    for c in range(h["n_colours"]):
        el = ebc[cp[c]:cp[c + 1]]
        nodes = mesh.tets[el].ravel()
        assert np.unique(nodes).size == nodes.size, f"colour {c} shares a node"
    # greedy colouring of a Kuhn mesh: a few dozen colours at most
    assert h["n_colours"] <= 64


def test_node_face_lists():
    mesh = synth.cube_mesh(3)
    h = build_host(mesh)
    for i in range(mesh.n_nodes):
        faces = h["nf_face"][h["nf_ptr"][i]:h["nf_ptr"][i + 1]]
        expect = np.nonzero((mesh.bfaces == i).any(axis=1))[0]
        np.testing.assert_array_equal(np.sort(faces), expect)


def test_setup_rejects_out_of_range_nodes():
    lib = L.load()
    tets = np.array([[0, 1, 2, 7]], np.int32)
    nnzb, ncb = C.c_int64(), C.c_int32()
    assert lib.vms_setup_sizes(4, 1, tets.ctypes.data, C.byref(nnzb), C.byref(ncb)) == -1
