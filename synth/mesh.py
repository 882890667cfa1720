"""Seeded synthetic tetrahedral meshes.

* ``cube_mesh(N, seed)``: the unit cube cut into N^3 hexahedra, each split
  into the six Kuhn simplices along its (0,0,0)-(1,1,1) diagonal.  Interior
  nodes are jittered by a seeded uniform perturbation of +-1% of the hex
  size; boundary nodes stay on their faces so the faces remain planar.
  The bottom face (z = 0) fixes the z velocity component; the top face
  (z = 1) carries a uniform dead traction (0, 0, t_top).
* ``tube_mesh(nr, nt, nz)``: a thick-walled tube (inner radius 1.0, wall 0.2,
  length 2.0) meshed structured in (r, theta, z), periodic in theta, with the
  same Kuhn split; carries two helical fibre directions per element.
* ``strip_mesh(nx, ny, nz)``: one eighth of the tensile-test strip of
  section 5.2 (10 x 3 x 0.5 mm), i.e. the box [0, 5] x [0, 1.5] x [0, 0.25] mm,
  with symmetry conditions on the three coordinate planes, the loading face
  x = 5 mm held to move along x only and loaded by a dead traction along x;
  two in-plane fibre families at +-phi from the loading direction.

Node numbering is lexicographic with the first index fastest (for the strip
the thickness index fastest and the length index slowest), tets are emitted
hex by hex in the same order, and every tet is positively oriented in the
reference configuration.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    name: str
    X: np.ndarray              # [n][3] float64 reference coordinates
    tets: np.ndarray           # [m][4] int32, positively oriented
    bfaces: np.ndarray         # [f][3] int32 loaded boundary triangles
    traction: np.ndarray       # [f][3] float64 dead traction at full load
    dir_mask: np.ndarray       # [n][4] uint8: 1 = Dirichlet on (vx, vy, vz, p)
    dir_vel: np.ndarray        # [n][3] float64 prescribed velocity on Dirichlet comps
    fibre: np.ndarray | None = None   # [m][2][3] float64 unit fibre directions
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])


# The six Kuhn simplices of a hex: one per ordering (a, b, c) of the axes,
# path 000 -> e_a -> e_a + e_b -> 111.
_PERMS = list(itertools.permutations(range(3)))


def _perm_sign(perm) -> int:
    s = 1
    p = list(perm)
    for i in range(3):
        for j in range(i + 1, 3):
            if p[i] > p[j]:
                s = -s
    return s


def _kuhn_tets(n1: int, n2: int, n3: int, node_id, wrap2: bool = False) -> np.ndarray:
    """Kuhn-split every hex of an n1 x n2 x n3 index grid.

    ``node_id(i, j, k)`` maps (vectorised) grid indices to node numbers.  With
    ``wrap2`` the second index is periodic.
    """
    i, j, k = np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij")
    # hex order: first index fastest
    i = i.transpose(2, 1, 0).ravel()
    j = j.transpose(2, 1, 0).ravel()
    k = k.transpose(2, 1, 0).ravel()
    base = np.stack([i, j, k], axis=1)
    out = []
    for perm in _PERMS:
        corners = [np.zeros(3, dtype=np.int64)]
        c = np.zeros(3, dtype=np.int64)
        for ax in perm:
            c = c.copy()
            c[ax] = 1
            corners.append(c)
        verts = []
        for c in corners:
            idx = base + c[None, :]
            jj = idx[:, 1] % n2 if wrap2 else idx[:, 1]
            verts.append(node_id(idx[:, 0], jj, idx[:, 2]))
        verts = np.stack(verts, axis=1)
        if _perm_sign(perm) < 0:           # odd ordering: swap to orient positively
            verts = verts[:, [0, 2, 1, 3]]
        out.append(verts)
    # interleave so tets of one hex are contiguous: [hex][6]
    tets = np.stack(out, axis=1).reshape(-1, 4)
    return tets.astype(np.int32)


def _faces_on(tets: np.ndarray, on_node: np.ndarray) -> np.ndarray:
    """Triangles of ``tets`` whose three vertices all satisfy ``on_node``."""
    faces = []
    for drop in range(4):
        keep = [a for a in range(4) if a != drop]
        f = tets[:, keep]
        sel = on_node[f].all(axis=1)
        faces.append(f[sel])
    return np.concatenate(faces, axis=0).astype(np.int32)


def cube_mesh(N: int, seed: int = 0, jitter: float = 0.01, t_top: float = -1.0e4) -> Mesh:
    """Unit cube, N^3 hexes x 6 Kuhn tets, seeded interior jitter."""
    n1 = N + 1
    g = np.arange(n1, dtype=np.float64) / N
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    X = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    ii = np.rint(X * N).astype(np.int64)
    interior = np.all((ii > 0) & (ii < N), axis=1)
    rng = np.random.default_rng(seed)
    h = 1.0 / N
    pert = rng.uniform(-jitter * h, jitter * h, size=X.shape)
    X = X + pert * interior[:, None]

    def node_id(i, j, k):
        return i + n1 * (j + n1 * k)

    tets = _kuhn_tets(N, N, N, node_id)
    top = ii[:, 2] == N
    bfaces = _faces_on(tets, top)
    traction = np.zeros((bfaces.shape[0], 3))
    traction[:, 2] = t_top
    dir_mask = np.zeros((X.shape[0], 4), dtype=np.uint8)
    dir_mask[ii[:, 2] == 0, 2] = 1
    dir_vel = np.zeros((X.shape[0], 3))
    return Mesh(name=f"cube{N}", X=X, tets=tets, bfaces=bfaces, traction=traction,
                dir_mask=dir_mask, dir_vel=dir_vel, fibre=None,
                meta={"N": N, "seed": seed, "jitter": jitter, "t_top": t_top})


def helical_fibres(X, tets, phi):
    """Fibre directions a_{1,2} = cos(phi) e_theta +- sin(phi) e_z at the element
    centroids and their derivatives with respect to phi (phi may be complex)."""
    cen = X[tets].mean(axis=1)
    ang = np.arctan2(cen[:, 1], cen[:, 0])
    e_t = np.stack([-np.sin(ang), np.cos(ang), np.zeros_like(ang)], axis=1)
    e_z = np.tile(np.array([0.0, 0.0, 1.0]), (tets.shape[0], 1))
    c, s = np.cos(phi), np.sin(phi)
    fibre = np.stack([c * e_t + s * e_z, c * e_t - s * e_z], axis=1)
    dfibre = np.stack([-s * e_t + c * e_z, -s * e_t - c * e_z], axis=1)
    return fibre, dfibre


def planar_fibres(n_tets, phi):
    """Fibre directions a_{1,2} = cos(phi) e_x +- sin(phi) e_y in every element
    and their derivatives with respect to phi (phi may be complex)."""
    c, s = np.cos(phi), np.sin(phi)
    one = np.ones(n_tets)
    zero = np.zeros(n_tets)
    fibre = np.stack([np.stack([c * one, s * one, zero], axis=1),
                      np.stack([c * one, -s * one, zero], axis=1)], axis=1)
    dfibre = np.stack([np.stack([-s * one, c * one, zero], axis=1),
                       np.stack([-s * one, -c * one, zero], axis=1)], axis=1)
    return fibre, dfibre


def fibre_field(mesh, phi):
    """The mesh's fibre field at fibre angle phi and its derivative in phi."""
    if mesh.meta.get("fibre_field") == "planar":
        return planar_fibres(mesh.n_tets, phi)
    return helical_fibres(mesh.X, mesh.tets, phi)


def tube_mesh(nr: int, nt: int, nz: int, r_in: float = 1.0, wall: float = 0.2,
              length: float = 2.0, fibre_deg: float = 45.0, stretch: float = 1.5,
              t_end: float = 1.0) -> Mesh:
    """Thick-walled tube, structured in (r, theta, z), theta periodic.

    z = 0 is clamped; on z = length the axial velocity is prescribed so that
    the axial stretch reaches ``stretch`` at ``t_end``; the other faces are
    traction free.  Fibres: cos(phi) e_theta +- sin(phi) e_z at the centroid.
    """
    r = r_in + wall * np.arange(nr + 1) / nr
    th = 2.0 * np.pi * np.arange(nt) / nt
    z = length * np.arange(nz + 1) / nz
    Z, T, R = np.meshgrid(z, th, r, indexing="ij")        # r fastest
    X = np.stack([(R * np.cos(T)).ravel(), (R * np.sin(T)).ravel(), Z.ravel()], axis=1)
    kz = np.repeat(np.arange(nz + 1), nt * (nr + 1))

    def node_id(i, j, k):
        return i + (nr + 1) * (j + nt * k)

    tets = _kuhn_tets(nr, nt, nz, node_id, wrap2=True)
    dir_mask = np.zeros((X.shape[0], 4), dtype=np.uint8)
    dir_vel = np.zeros((X.shape[0], 3))
    dir_mask[kz == 0, 0:3] = 1
    dir_mask[kz == nz, 2] = 1
    dir_vel[kz == nz, 2] = (stretch - 1.0) * length / t_end
    fibre, _ = helical_fibres(X, tets, np.deg2rad(fibre_deg))
    bfaces = np.zeros((0, 3), dtype=np.int32)
    traction = np.zeros((0, 3))
    return Mesh(name=f"tube{nr}x{nt}x{nz}", X=X, tets=tets, bfaces=bfaces,
                traction=traction, dir_mask=dir_mask, dir_vel=dir_vel, fibre=fibre,
                meta={"nr": nr, "nt": nt, "nz": nz, "stretch": stretch, "t_end": t_end,
                      "fibre_rad": float(np.deg2rad(fibre_deg)), "fibre_field": "helical"})


# Dimensions of the tensile specimen of section 5.2 in metres; the model is
# the eighth x, y, z >= 0 of the specimen centred at the origin.
STRIP_FULL = (10.0e-3, 3.0e-3, 0.5e-3)


def strip_dims(n: int):
    """Hexes per axis of the eighth-strip for mesh size dx = 1/n of its
    half-length (the paper's 1/dx = 200, 400, 600 ladder): n x 0.3n x 0.05n."""
    return n, max(1, int(round(0.3 * n))), max(1, int(round(0.05 * n)))


def strip_mesh(nx: int, ny: int, nz: int, fibre_deg: float = 49.98, force: float = 2.0,
               seed: int = 0, jitter: float = 0.01) -> Mesh:
    """Eighth of the tensile strip, nx * ny * nz hexes x 6 Kuhn tets.

    Symmetry planes fix u_x on x = 0, u_y on y = 0 and u_z on z = 0.  The
    loading face x = L/2 moves along x only (u_y = u_z = 0 there) and carries
    the dead traction force / (W T) along x, the nominal stress of the full
    specimen under the tensile force.  Interior nodes get a seeded jitter of
    +-1% of the hex size per axis; boundary nodes stay on their planes.
    """
    lx, ly, lz = (0.5 * d for d in STRIP_FULL)
    gx = lx * np.arange(nx + 1) / nx
    gy = ly * np.arange(ny + 1) / ny
    gz = lz * np.arange(nz + 1) / nz
    # nodes numbered with the thickness index fastest and the length index
    # slowest: the narrowest bandwidth of the node graph for this shape
    xx, yy, zz = np.meshgrid(gx, gy, gz, indexing="ij")
    X = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    ix, iy, iz = (a.ravel() for a in np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1),
                                                  indexing="ij"))
    interior = (ix > 0) & (ix < nx) & (iy > 0) & (iy < ny) & (iz > 0) & (iz < nz)
    h = np.array([lx / nx, ly / ny, lz / nz])
    rng = np.random.default_rng(seed)
    pert = rng.uniform(-1.0, 1.0, size=X.shape) * (jitter * h)[None, :]
    X = X + pert * interior[:, None]

    def node_id(a, b, c):          # a: z index, b: y index, c: x index
        return a + (nz + 1) * (b + (ny + 1) * c)

    # hexes in the same order (z fastest); the (z, y, x) index frame is a
    # reflection of (x, y, z), so every simplex is reoriented
    tets = _kuhn_tets(nz, ny, nx, node_id)[:, [0, 2, 1, 3]]
    load = ix == nx
    bfaces = _faces_on(tets, load)
    t_full = force / (STRIP_FULL[1] * STRIP_FULL[2])
    traction = np.zeros((bfaces.shape[0], 3))
    traction[:, 0] = t_full
    dir_mask = np.zeros((X.shape[0], 4), dtype=np.uint8)
    dir_mask[ix == 0, 0] = 1
    dir_mask[iy == 0, 1] = 1
    dir_mask[iz == 0, 2] = 1
    dir_mask[load, 1] = 1
    dir_mask[load, 2] = 1
    dir_vel = np.zeros((X.shape[0], 3))
    phi = float(np.deg2rad(fibre_deg))
    fibre, _ = planar_fibres(tets.shape[0], phi)
    return Mesh(name=f"strip{nx}x{ny}x{nz}", X=X, tets=tets, bfaces=bfaces, traction=traction,
                dir_mask=dir_mask, dir_vel=dir_vel, fibre=fibre,
                meta={"nx": nx, "ny": ny, "nz": nz, "seed": seed, "jitter": jitter, "force": force,
                      "t_full": t_full, "fibre_rad": phi, "fibre_field": "planar"})
