"""Krylov solvers and exact block preconditioners (section 4), oracle.

``fgmres`` is textbook flexible GMRES (Arnoldi by modified Gram-Schmidt,
Givens rotations on the Hessenberg matrix, x0 = 0, no restart), stopping when
the least-squares residual |g_{j+1}| <= max(rtol * ||b||, atol).  With the
identity preconditioner it is plain GMRES.

``block_preconditioner`` applies the block factorization of
[[A, B], [C, D]] with exact solves: the full LDU form is the Schur complement
reduction of Algorithm 1; 'upper' (DU), 'lower' (LD) and 'diag' (D) use part
of the factorization (the remark on partial factorizations).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def fgmres(matvec, b, precond=None, rtol=1e-10, atol=1e-50, maxit=200):
    b = np.asarray(b, dtype=float)
    n = b.shape[0]
    beta = float(np.linalg.norm(b))
    x = np.zeros(n)
    if beta == 0.0:
        return x, 0, [0.0]
    V = np.zeros((maxit + 1, n))
    Z = np.zeros((maxit, n))
    Hm = np.zeros((maxit + 1, maxit))
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    V[0] = b / beta
    hist = [beta]
    tol = max(rtol * beta, atol)
    k = 0
    for j in range(maxit):
        Z[j] = precond(V[j]) if precond is not None else V[j]
        w = matvec(Z[j])
        for i in range(j + 1):                       # modified Gram-Schmidt
            Hm[i, j] = np.dot(w, V[i])
            w = w - Hm[i, j] * V[i]
        Hm[j + 1, j] = np.linalg.norm(w)
        for i in range(j):                           # apply previous rotations
            t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
            Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
            Hm[i, j] = t
        den = np.hypot(Hm[j, j], Hm[j + 1, j])
        cs[j], sn[j] = Hm[j, j] / den, Hm[j + 1, j] / den
        Hm[j, j] = den
        Hm[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        hist.append(abs(g[j + 1]))
        k = j + 1
        if abs(g[j + 1]) <= tol or Hm[j, j] == 0.0:
            break
        hn = np.linalg.norm(w)
        if hn == 0.0:
            break
        V[j + 1] = w / hn
    y = sla.solve_triangular(Hm[:k, :k], g[:k])
    x = Z[:k].T @ y
    return x, k, hist


def schur_dense(A, B, C, D):
    """S = D - C A^-1 B formed densely (small meshes only)."""
    luA = spla.splu(A.tocsc())
    AinvB = luA.solve(B.toarray())
    return D.toarray() - C @ AinvB


def block_preconditioner(A, B, C, D, variant="ldu"):
    """Exact block preconditioner P^-1 r for r = [r_v; r_p] (split ordering)."""
    luA = spla.splu(A.tocsc())
    S = schur_dense(A, B, C, D)
    luS = sla.lu_factor(S)
    nv = A.shape[0]

    def apply(r):
        rv, rp = r[:nv].copy(), r[nv:].copy()
        if variant == "ldu":                          # Algorithm 1
            xh = luA.solve(rv)
            rp = rp - C @ xh
            xp = sla.lu_solve(luS, rp)
            rv = rv - B @ xp
            xv = luA.solve(rv)
        elif variant == "upper":
            xp = sla.lu_solve(luS, rp)
            xv = luA.solve(rv - B @ xp)
        elif variant == "lower":
            xv = luA.solve(rv)
            xp = sla.lu_solve(luS, rp - C @ xv)
        elif variant == "diag":
            xv = luA.solve(rv)
            xp = sla.lu_solve(luS, rp)
        else:
            raise ValueError(variant)
        return np.concatenate([xv, xp])

    return apply


def shat(A, B, C, D):
    """S^ = D - C diag(A)^-1 B (section 4.2), sparse."""
    return (D - C @ sp.diags(1.0 / A.diagonal()) @ B).tocsr()


def simple_preconditioner(A, B, C, D):
    """P_SIMPLE^-1 r with exact solves of A and S^ (section 4.3, H1 = H2 =
    diag(A)^-1): P_SIMPLE = L Dg U with L = [[I, 0], [C A^-1, I]],
    Dg = diag(A, S^), U = [[I, diag(A)^-1 B], [0, I]], inverted factor by
    factor: y_v = A^-1 r_v, y_p = S^-1 (r_p - C y_v), x_v = y_v - diag(A)^-1 B y_p."""
    luA = spla.splu(A.tocsc())
    luS = spla.splu(shat(A, B, C, D).tocsc())
    dAinv = 1.0 / A.diagonal()
    nv = A.shape[0]

    def apply(r):
        rv, rp = r[:nv], r[nv:]
        yv = luA.solve(rv)
        xp = luS.solve(rp - C @ yv)
        xv = yv - dAinv * (B @ xp)
        return np.concatenate([xv, xp])

    return apply


def schur_apply_matrix_free(A, B, C, D, xp):
    """Algorithm 2 with an exact inner solve: D x_p - C A^-1 (B x_p)."""
    xh = D @ xp
    xb = B @ xp
    xt = spla.spsolve(A.tocsc(), xb)
    return xh - C @ xt
