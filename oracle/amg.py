"""Aggregation AMG for the momentum-block solves, oracle (TEST INFRASTRUCTURE).

The paper preconditions every A-solve by algebraic multigrid (BoomerAMG, with
the settings of its section 5 table); the GPU path replaces it by its own
plain-aggregation multigrid, and this module is that method written out with
NumPy/SciPy so the GPU hierarchy and V-cycle can be checked against it.  It
shares no code with the HIP path and nothing here is imported by it.

The method (aggregation multigrid after Vanek, Mandel and Brezina 1996, without
prolongator smoothing):

1. Aggregates.  Greedy, in node order, on the graph of the level (fine level:
   nodes coupled by a tetrahedron):
   (1) a node whose whole neighbourhood is free forms an aggregate of that
       neighbourhood;
   (2) every node still free joins the aggregate of its first neighbour (in
       increasing index) that phase 1 placed;
   (3) a node still free forms an aggregate with its free neighbours.
2. Near-null space.  The A-block of the velocity is a mass matrix plus
   (alpha_f gamma dt)^2/alpha_m times the linearised isochoric stiffness, whose
   kernel is the conformal motions: 3 translations, 3 rotations, the dilation
   and 3 special conformal fields 2 (a.y) y - |y|^2 a.  Per aggregate they are
   evaluated at y = (X - c)/h (c the centroid of its nodes, h the largest
   |X - c| component, 1 if zero), zeroed on Dirichlet components.
3. Tentative prolongator.  Per aggregate, modified Gram-Schmidt of those 10
   columns over the aggregate's rows (nodes ascending, dofs in order); a column
   whose remainder is at most 1e-10 of its norm is dropped (zero column).
   B = Q R per aggregate; the coarse near-null space is R (rows = the 10 coarse
   dofs of the aggregate).  In the scaled system x = W x* the prolongator is
   P* = W^-1 Q (W of the velocity dofs), so the coarse operator does not
   depend on W: P*^T (W A W) P* = Q^T A Q.
4. Coarse operator A_c = P^T A P, with a unit diagonal on dropped coarse dofs.
5. Smoother.  Chebyshev iteration on D^-1 A (D the block diagonal: 3x3 on the
   finest level, 10x10 on coarse ones) over [lmax/30, lmax]; lmax is 1.1 times
   the ratio ||D^-1 A x|| / ||x|| after 12 power steps from a SplitMix64 vector.
6. V-cycle: degree-k pre-smoothing from zero, residual, restriction P^T,
   recursion, prolongation, degree-k post-smoothing; on the coarsest level
   degree k_c smoothing from zero only.  The levels between the finest and
   the coarsest may take their own degree k_m in place of k.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

NMODES = 10
DROP_TOL = 1e-10
POWER_STEPS = 12
LMAX_SAFETY = 1.1
CHEB_RATIO = 30.0

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def splitmix64_raw(seed: int, i: int) -> int:
    """Output i (from 0) of SplitMix64 started at state `seed`, as a 64-bit integer."""
    z = (seed + (i + 1) * _GOLDEN) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def splitmix64(seed: int, n: int) -> np.ndarray:
    """n values in [-1, 1): output i of the SplitMix64 generator (Steele, Lea
    and Flood 2014) started at `seed`, i.e. the mix of seed + (i+1) * golden
    gamma, top 53 bits as a fraction."""
    out = np.empty(n)
    for i in range(n):
        out[i] = 2.0 * ((splitmix64_raw(seed, i) >> 11) * 2.0 ** -53) - 1.0
    return out


def aggregate(ptr: np.ndarray, idx: np.ndarray):
    """Greedy three-phase aggregation of the graph (CSR ptr/idx, self loops
    allowed).  Returns (agg[n], n_agg)."""
    n = len(ptr) - 1
    agg = np.full(n, -1, dtype=np.int64)
    na = 0
    for i in range(n):                                   # phase 1
        nb = idx[ptr[i]:ptr[i + 1]]
        if agg[i] < 0 and np.all(agg[nb] < 0):
            agg[nb] = na
            agg[i] = na
            na += 1
    phase1 = agg.copy()
    for i in range(n):                                   # phase 2
        if agg[i] >= 0:
            continue
        for j in np.sort(idx[ptr[i]:ptr[i + 1]]):
            if j != i and phase1[j] >= 0:
                agg[i] = phase1[j]
                break
    for i in range(n):                                   # phase 3
        if agg[i] >= 0:
            continue
        agg[i] = na
        for j in np.sort(idx[ptr[i]:ptr[i + 1]]):
            if agg[j] < 0:
                agg[j] = na
        na += 1
    return agg, na


def members(agg: np.ndarray, na: int):
    """Nodes of each aggregate, ascending."""
    order = np.argsort(agg, kind="stable")
    starts = np.searchsorted(agg[order], np.arange(na + 1))
    return [order[starts[a]:starts[a + 1]] for a in range(na)]


def conformal_modes(Y: np.ndarray) -> np.ndarray:
    """[k][3][10] velocity fields at points Y[k]: translations, rotations,
    dilation and the special conformal fields."""
    k = Y.shape[0]
    B = np.zeros((k, 3, NMODES))
    for d in range(3):
        B[:, d, d] = 1.0
    x, y, z = Y[:, 0], Y[:, 1], Y[:, 2]
    B[:, 1, 3], B[:, 2, 3] = -z, y           # rotation about e_x
    B[:, 0, 4], B[:, 2, 4] = z, -x           # about e_y
    B[:, 0, 5], B[:, 1, 5] = -y, x           # about e_z
    B[:, :, 6] = Y                           # dilation
    s2 = np.sum(Y * Y, axis=1)
    for a in range(3):
        B[:, :, 7 + a] = 2.0 * Y[:, a:a + 1] * Y
        B[:, a, 7 + a] -= s2
    return B


def mgs_drop(M: np.ndarray):
    """Modified Gram-Schmidt of the columns of M with the drop rule; returns
    (Q, R) with M = Q R (dropped columns: zero in Q, zero row in R)."""
    rows, k = M.shape
    Q = np.zeros((rows, k))
    R = np.zeros((k, k))
    for j in range(k):
        v = M[:, j].copy()
        n0 = np.linalg.norm(v)
        for i in range(j):
            if R[i, i] == 0.0:
                continue
            R[i, j] = Q[:, i] @ v
            v -= R[i, j] * Q[:, i]
        nv = np.linalg.norm(v)
        if n0 > 0.0 and nv > DROP_TOL * n0:
            R[j, j] = nv
            Q[:, j] = v / nv
    return Q, R


def tentative(mem, B: np.ndarray, blk: int):
    """Prolongator Q (n*blk x na*10, CSR), coarse near-null space R
    (na*10 x 10) and the dropped-dof mask of the coarse level."""
    na = len(mem)
    rows, cols, vals = [], [], []
    Rc = np.zeros((na * NMODES, NMODES))
    dropped = np.zeros(na * NMODES, dtype=bool)
    n = sum(len(m) for m in mem)
    for a, nodes in enumerate(mem):
        dofs = (nodes[:, None] * blk + np.arange(blk)).ravel()
        Q, R = mgs_drop(B[dofs])
        rows.append(np.repeat(dofs, NMODES))
        cols.append(np.tile(a * NMODES + np.arange(NMODES), dofs.size))
        vals.append(Q.ravel())
        Rc[a * NMODES:(a + 1) * NMODES] = R
        dropped[a * NMODES:(a + 1) * NMODES] = np.diag(R) == 0.0
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n * blk, na * NMODES))
    return P, Rc, dropped


def fine_modes(X: np.ndarray, mem, dir_vel: np.ndarray) -> np.ndarray:
    """Unscaled near-null space of the finest level, [3n][10], per aggregate
    centred and scaled, zero on Dirichlet components (dir_vel: bool [n][3])."""
    n = X.shape[0]
    B = np.zeros((n, 3, NMODES))
    for nodes in mem:
        Xa = X[nodes]
        c = Xa.mean(axis=0)
        h = np.abs(Xa - c).max()
        h = h if h > 0.0 else 1.0
        B[nodes] = conformal_modes((Xa - c) / h)
    B[dir_vel] = 0.0
    return B.reshape(3 * n, NMODES)


def block_diag_inv(A: sp.spmatrix, blk: int) -> sp.csr_matrix:
    """Inverse of the blk x blk diagonal blocks of A (a block with a zero row
    gets a unit diagonal there)."""
    n = A.shape[0] // blk
    Ac = A.tocoo()
    D = np.zeros((n, blk, blk))
    m = (Ac.row // blk) == (Ac.col // blk)
    np.add.at(D, (Ac.row[m] // blk, Ac.row[m] % blk, Ac.col[m] % blk), Ac.data[m])
    for i in range(n):
        for q in np.where(np.all(D[i] == 0.0, axis=1))[0]:
            D[i, q, q] = 1.0
    return sp.block_diag(list(np.linalg.inv(D)), format="csr")


def power_lmax(A, Dinv, seed: int) -> float:
    """LMAX_SAFETY times ||D^-1 A x_k|| / ||x_k|| after POWER_STEPS steps of the
    power method on D^-1 A from the SplitMix64 vector of `seed`."""
    x = splitmix64(seed, A.shape[0])
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(POWER_STEPS):
        y = Dinv @ (A @ x)
        lam = np.linalg.norm(y)
        x = y / lam
    return LMAX_SAFETY * lam


class Level:
    pass


def mesh_graph(tets: np.ndarray, n: int) -> sp.csr_matrix:
    """Node graph of a tetrahedral mesh: nodes coupled by a tetrahedron (with self loops)."""
    r = np.repeat(tets, 4, axis=1).ravel()
    c = np.tile(tets, (1, 4)).ravel()
    G = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(n, n)).tocsr()
    G.sum_duplicates()
    G.data[:] = 1.0
    return G


def graph_of(A: sp.spmatrix, blk: int) -> sp.csr_matrix:
    """Node graph of a block matrix (nodes = blk-dof groups)."""
    C = A.tocoo()
    n = A.shape[0] // blk
    G = sp.coo_matrix((np.ones(C.nnz), (C.row // blk, C.col // blk)), shape=(n, n)).tocsr()
    G.sum_duplicates()
    G.data[:] = 1.0
    return G


def build(A: sp.spmatrix, W: np.ndarray, X: np.ndarray, dir_vel: np.ndarray, max_levels: int = 4,
          min_coarse: int = 64, graph: sp.spmatrix | None = None):
    """Hierarchy for the scaled velocity block A* = W A W ([3n x 3n], dofs
    node-interleaved); W: [n][3] scaling of the velocity dofs; X: [n][3];
    dir_vel: bool [n][3].  Coarsening stops at max_levels levels or when a
    level has at most min_coarse nodes.  `graph` defaults to A*'s node graph."""
    n = X.shape[0]
    G = graph if graph is not None else graph_of(A, 3)
    levels = []
    Acur, blk = sp.csr_matrix(A), 3
    B = None
    for lev in range(max_levels):
        L = Level()
        L.A, L.blk = Acur, blk
        L.Dinv = block_diag_inv(L.A, blk)
        L.lmax = power_lmax(L.A, L.Dinv, seed=lev + 1)
        levels.append(L)
        nn = L.A.shape[0] // blk
        if lev == max_levels - 1 or nn <= min_coarse:
            break
        G = G.tocsr()
        agg, na = aggregate(G.indptr, G.indices)
        mem = members(agg, na)
        L.agg, L.mem = agg, mem
        if lev == 0:
            B = fine_modes(X, mem, dir_vel)
        Q, R, dropped = tentative(mem, B, blk)
        L.Q = Q
        # scaled system: P* = W^-1 Q on the finest level
        L.P = (sp.diags(1.0 / W.ravel()) @ Q).tocsr() if lev == 0 else Q
        Ac = (L.P.T @ L.A @ L.P).tocsr()
        Ac = (Ac + sp.diags(dropped.astype(float))).tocsr()
        L.dropped_next = dropped
        Pa = sp.csr_matrix((np.ones(nn), (np.arange(nn), agg)), shape=(nn, na))
        G = (Pa.T @ G @ Pa).tocsr()
        G.data[:] = 1.0
        Acur, blk, B = Ac, NMODES, R
    return levels


def chebyshev(L, b: np.ndarray, x: np.ndarray | None, degree: int) -> np.ndarray:
    """degree steps of the Chebyshev iteration for L.A x = b preconditioned by
    L.Dinv on [lmax/CHEB_RATIO, lmax], from x (None: zero)."""
    lmax = L.lmax
    lmin = lmax / CHEB_RATIO
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    if x is None:
        x = np.zeros_like(b)
        r = L.Dinv @ b
    else:
        x = x.copy()
        r = L.Dinv @ (b - L.A @ x)
    d = r / theta
    for k in range(degree):
        x = x + d
        if k == degree - 1:
            break
        r = r - L.Dinv @ (L.A @ d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * r
        rho = rho_new
    return x


def vcycle(levels, b: np.ndarray, degree: int = 2, coarse_degree: int = 8, lev: int = 0,
           coarse_solve=None, mid_degree: int = 0) -> np.ndarray:
    """One V-cycle for levels[lev].A x = b from x = 0.  coarse_solve(A, b)
    replaces the coarsest smoothing when given (used by the pins).  The levels
    between the finest and the coarsest smooth with mid_degree steps (0: degree)."""
    L = levels[lev]
    if lev == len(levels) - 1:
        if coarse_solve is not None:
            return coarse_solve(L.A, b)
        return chebyshev(L, b, None, coarse_degree)
    k = degree if lev == 0 or mid_degree == 0 else mid_degree
    x = chebyshev(L, b, None, k)
    r = b - L.A @ x
    e = vcycle(levels, L.P.T @ r, degree, coarse_degree, lev + 1, coarse_solve, mid_degree)
    x = x + L.P @ e
    return chebyshev(L, b, x, k)


def pcg(A, b: np.ndarray, M, rtol: float, maxit: int = 1000):
    """Preconditioned CG from x = 0, stopping on ||r|| <= rtol ||b||; returns (x, iterations)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = r @ z
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0
    for k in range(1, maxit + 1):
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        if np.linalg.norm(r) <= rtol * nb:
            return x, k
        z = M(r)
        rzn = r @ z
        p = z + (rzn / rz) * p
        rz = rzn
    return x, maxit
