"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/vms.h declares, and its integer setup (block
pattern, transpose map, block contribution lists, node->face lists) is exact
against independent constructions."""
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
    nnzb, sw, w2, span = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
    assert lib.vms_setup_sizes(n, m, tets.ctypes.data, C.byref(nnzb), C.byref(sw), C.byref(w2), C.byref(span)) == 0
    nz = nnzb.value
    assert nz == sw.value * n and sw.value % 16 == 0
    assert w2.value % 64 == 0
    h = {"W": sw.value, "W2": w2.value, "span": span.value, "row_len": np.zeros(n, np.int32),
         "col": np.zeros(nz, np.int32), "tpos": np.zeros(nz, np.int32),
         "diag_pos": np.zeros(n, np.int32), "blk_src_ptr": np.zeros(nz + 1, np.int32),
         "blk_src": np.zeros(16 * m, np.int32),
         "shat_col": np.zeros(n * w2.value, np.int32), "shat_off": np.zeros(n * w2.value, np.int16),
         "nf_ptr": np.zeros(n + 1, np.int32), "nf_face": np.zeros(max(3 * f, 1), np.int32)}
    rc = lib.vms_setup_build(n, m, tets.ctypes.data, f, bf.ctypes.data,
                             *(h[k].ctypes.data for k in ("row_len", "col", "tpos", "diag_pos", "blk_src_ptr",
                                                          "blk_src", "shat_col", "shat_off", "nf_ptr", "nf_face")))
    assert rc == 0
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
    W = h["W"]
    np.testing.assert_array_equal(h["row_len"], np.diff(G.indptr))
    assert W == 16 * ((np.diff(G.indptr).max() + 15) // 16)
    col = h["col"]
    rows = np.repeat(np.arange(n), W)
    slot = np.arange(n * W) % W
    real = slot < np.repeat(h["row_len"], W)
    # real slots: the sorted CSR columns of the row; padding slots: the row's own node, mapped to themselves
    np.testing.assert_array_equal(col[real], G.indices)
    np.testing.assert_array_equal(col[~real], rows[~real])
    np.testing.assert_array_equal(h["tpos"][~real], np.nonzero(~real)[0])
    # transpose map and diagonal positions
    tp = h["tpos"][real]
    assert np.all(real[tp])
    np.testing.assert_array_equal(rows[tp], col[real])
    np.testing.assert_array_equal(col[tp], rows[real])
    np.testing.assert_array_equal(col[h["diag_pos"]], np.arange(n))
    np.testing.assert_array_equal(rows[h["diag_pos"]], np.arange(n))
    assert np.all(real[h["diag_pos"]])
    # block contribution lists: every element-local pair exactly once, under its block, in element order
    ptr, src = h["blk_src_ptr"], h["blk_src"]
    assert ptr[0] == 0 and ptr[-1] == 16 * mesh.n_tets
    np.testing.assert_array_equal(np.sort(src), np.arange(16 * mesh.n_tets))
    blk = np.repeat(np.arange(col.size), np.diff(ptr))
    e, a, b = src >> 4, (src >> 2) & 3, src & 3
    np.testing.assert_array_equal(rows[blk], t[e, a])
    np.testing.assert_array_equal(col[blk], t[e, b])
    for k in range(col.size):
        assert np.all(np.diff(e[ptr[k]:ptr[k + 1]]) >= 0)
    assert np.all(np.diff(ptr)[~real] == 0)      # padding slots receive nothing
    # distance-2 pattern: the off-diagonal pattern of G @ G (nodes two graph steps away), sorted, in W2 slots
    G2 = (G @ G).tocsr()
    G2.setdiag(0)
    G2.eliminate_zeros()
    G2.sort_indices()
    W2 = h["W2"]
    assert W2 == 64 * ((np.diff(G2.indptr).max() + 63) // 64)
    sc = h["shat_col"].reshape(n, W2)
    for i in range(n):
        real = G2.indices[G2.indptr[i]:G2.indptr[i + 1]]
        np.testing.assert_array_equal(sc[i, :real.size], real)
        assert np.all(sc[i, real.size:] == i)
    # a diagonal block lists each element around its node once, with pair a*4 + a
    d = h["diag_pos"]
    for i in range(n):
        s_ = src[ptr[d[i]]:ptr[d[i] + 1]]
        assert np.all((s_ & 15) % 5 == 0)
        np.testing.assert_array_equal(s_ >> 4, np.nonzero((t == i).any(axis=1))[0])


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
    nnzb, sw, w2 = C.c_int64(), C.c_int32(), C.c_int32()
    assert lib.vms_setup_sizes(4, 1, tets.ctypes.data, C.byref(nnzb), C.byref(sw), C.byref(w2), None) == -1


def _sizes(n, tets):
    lib = L.load()
    tets = np.ascontiguousarray(tets, np.int32).reshape(-1, 4)
    nnzb, sw, w2 = C.c_int64(), C.c_int32(), C.c_int32()
    rc = lib.vms_setup_sizes(n, tets.shape[0], tets.ctypes.data, C.byref(nnzb), C.byref(sw), C.byref(w2), None)
    return rc, nnzb.value, sw.value, w2.value


def test_setup_isolated_nodes_and_empty_mesh():
    """Nodes outside every element keep a diagonal block (no contributions, empty distance-2 row);
    a mesh with no elements has only such rows."""
    mesh = synth.cube_mesh(1)
    n0 = mesh.n_nodes
    X = np.vstack([mesh.X, [[5.0, 5.0, 5.0], [6.0, 6.0, 6.0]]])
    m2 = type(mesh)(**{**mesh.__dict__, "X": X, "dir_mask": np.zeros((n0 + 2, 4), np.uint8),
                       "dir_vel": np.zeros((n0 + 2, 3))})
    h = build_host(m2)
    W = h["W"]
    for i in (n0, n0 + 1):
        assert h["row_len"][i] == 1
        np.testing.assert_array_equal(h["col"][W * i:W * i + W], i)
        assert h["diag_pos"][i] == W * i
        b = h["diag_pos"][i]
        assert h["blk_src_ptr"][b + 1] == h["blk_src_ptr"][b]
        np.testing.assert_array_equal(h["shat_col"].reshape(-1, h["W2"])[i], i)
    rc, nnzb, sw, w2 = _sizes(3, np.zeros((0, 4), np.int32))
    assert rc == 0 and sw == 16 and nnzb == 48 and w2 == 64


def test_setup_limits():
    """n_tets beyond VMS_MAX_TETS is refused before the array is read; a distance-2 row longer
    than VMS_MAX_SHAT_ROW (here: every node couples to a hub node) is refused."""
    lib = L.load()
    small = np.zeros(4, np.int32)
    nnzb, sw, w2 = C.c_int64(), C.c_int32(), C.c_int32()
    assert lib.vms_setup_sizes(4, 134217728, small.ctypes.data, C.byref(nnzb), C.byref(sw), C.byref(w2), None) == -1
    assert lib.vms_setup_sizes(4, -1, small.ctypes.data, C.byref(nnzb), C.byref(sw), C.byref(w2), None) == -1
    assert lib.vms_setup_sizes(4, 1, small.ctypes.data, None, C.byref(sw), C.byref(w2), None) == -1
    hub = np.array([[0, 3 * k + 1, 3 * k + 2, 3 * k + 3] for k in range(66)], np.int32)
    rc, nnzb_, sw_, w2_ = _sizes(199, hub)
    assert rc == -1
    few = hub[:20]                     # 61 nodes: the longest distance-2 row has 60 entries
    rc, nnzb_, sw_, w2_ = _sizes(61, few)
    assert rc == 0 and sw_ == 64 and w2_ == 64 and nnzb_ == 64 * 61


@pytest.mark.parametrize("N", [2, 4])
def test_shat_offsets_and_span(N):
    """shat_off is shat_col minus the row (padding slots: 0), and the span
    reported by vms_setup_sizes is the largest |offset|."""
    mesh = synth.cube_mesh(N)
    h = build_host(mesh)
    n, W2 = mesh.n_nodes, h["W2"]
    off = h["shat_col"].reshape(n, W2) - np.arange(n)[:, None]
    np.testing.assert_array_equal(h["shat_off"].reshape(n, W2), off)
    assert h["span"] == np.abs(off).max()


def test_shat_offsets_refused_when_too_far():
    """A tet joining nodes 40000 apart: the span says so, and building the
    2-byte offsets is refused (the caller then passes NULL); without them the
    build succeeds."""
    lib = L.load()
    n = 40001
    tets = np.array([[0, 1, 2, 40000]], np.int32)
    nnzb, sw, w2, span = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
    assert lib.vms_setup_sizes(n, 1, tets.ctypes.data, C.byref(nnzb), C.byref(sw), C.byref(w2), C.byref(span)) == 0
    assert span.value == 40000
    nz = nnzb.value
    arrs = [np.zeros(n, np.int32), np.zeros(nz, np.int32), np.zeros(nz, np.int32), np.zeros(n, np.int32),
            np.zeros(nz + 1, np.int32), np.zeros(16, np.int32), np.zeros(n * w2.value, np.int32)]
    off = np.zeros(n * w2.value, np.int16)
    tail = [np.zeros(n + 1, np.int32), np.zeros(1, np.int32)]
    args = [a.ctypes.data for a in arrs]
    assert lib.vms_setup_build(n, 1, tets.ctypes.data, 0, None, *args, off.ctypes.data,
                               *[a.ctypes.data for a in tail]) == -1
    assert lib.vms_setup_build(n, 1, tets.ctypes.data, 0, None, *args, None, *[a.ctypes.data for a in tail]) == 0


def test_noalloc_scratch_size_and_limit():
    """The static scratch of vms_step_noalloc is 64 MiB; the default solver
    options fit an 8^3 cube's time step in it and not a 12^3 one (the entry
    point refuses the latter before launching anything)."""
    lib = L.load()
    assert lib.vms_noalloc_scratch_bytes() == 64 << 20
    from paper_1809_06350_amd import vms as V
    for N, fits in ((8, True), (12, False)):
        mesh = L.Mesh()
        mesh.n_nodes, mesh.n_tets, mesh.slot_width = (N + 1) ** 3, 6 * N ** 3, 16
        mesh.nnzb, mesh.shat_width = 16 * (N + 1) ** 3, 64
        need = lib.vms_step_workspace(C.byref(mesh), C.byref(V.solver_opts()))
        assert (need <= lib.vms_noalloc_scratch_bytes()) == fits
