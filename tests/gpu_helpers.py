"""Shared helpers of the GPU parity tests (format conversion only)."""
import numpy as np
import scipy.sparse as sp
import torch


def pattern(prob):
    """(row of every block slot, its column, mask of the real (non-padding) slots)."""
    h = prob.host
    n, W = prob.mesh.n_nodes, prob.slot_width
    rows = np.repeat(np.arange(n), W)
    real = (np.arange(n * W) % W) < np.repeat(h["row_len"], W)
    return rows, h["col"], real


def blocks_from_scipy(prob, K):
    """Entry-major block arrays of an interleaved 4n x 4n matrix on prob's pattern (padding slots zero)."""
    rows, col, real = pattern(prob)
    rows = np.where(real, rows, 0)
    col = np.where(real, col, 0)
    K = K.tocsr()
    A = np.zeros((9, col.size))
    B = np.zeros((3, col.size))
    Cm = np.zeros((3, col.size))
    for r in range(3):
        for c in range(3):
            A[3 * r + c] = np.asarray(K[4 * rows + r, 4 * col + c]).ravel()
        B[r] = np.asarray(K[4 * rows + r, 4 * col + 3]).ravel()
        Cm[r] = np.asarray(K[4 * rows + 3, 4 * col + r]).ravel()
    D = np.asarray(K[4 * rows + 3, 4 * col + 3]).ravel()
    for arr in (A, B, Cm):
        arr[:, ~real] = 0.0
    D[~real] = 0.0
    return A, B, Cm, D


def scipy_from_blocks(prob, A, B, Cm, D):
    n = prob.mesh.n_nodes
    rows, col, real = pattern(prob)
    rows, col = rows[real], col[real]
    A, B, Cm, D = A[:, real], B[:, real], Cm[:, real], D[real]
    R, Cc, V = [], [], []
    for r in range(3):
        for c in range(3):
            R.append(4 * rows + r); Cc.append(4 * col + c); V.append(A[3 * r + c])
        R.append(4 * rows + r); Cc.append(4 * col + 3); V.append(B[r])
        R.append(4 * rows + 3); Cc.append(4 * col + r); V.append(Cm[r])
    R.append(4 * rows + 3); Cc.append(4 * col + 3); V.append(D)
    return sp.coo_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(Cc))),
                         shape=(4 * n, 4 * n)).tocsr()


def gpu_K_scipy(prob, K):
    return scipy_from_blocks(prob, *(t.double().cpu().numpy() for t in (K.A, K.B, K.C, K.D)))


def upload_K(prob, Ksp):
    K = prob.new_matrix()
    for t, a in zip((K.A, K.B, K.C, K.D), blocks_from_scipy(prob, Ksp)):
        t.copy_(torch.from_numpy(a))
    return K


def rel_err(a, b):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
