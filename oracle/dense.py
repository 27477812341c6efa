"""Dense FP64 constructions for tiny images.  TEST INFRASTRUCTURE ONLY.

These build the paper's matrices explicitly (S, B-bar, W-hat, A) from their
definitions, independently of the matrix-free oracle in ``bilateral.py``, so
that tests can pin the oracle against the paper: the pixel-space loss
(Eq. pixel_loss), the factorisation W-hat = S^T D_m^-1 D_n B D_n D_m^-1 S
(Eq. equiv), the bilateral-space quadratic (Eq. quad_min) and its solution
(Eq. solution).  Sizes are O(P^2) and O(V^2): keep P below a few hundred.
"""
from __future__ import annotations

import numpy as np


def splat_matrix(idx: np.ndarray, V: int) -> np.ndarray:
    """S as a dense V x P matrix: S[v, p] = 1 iff pixel p lies on vertex v."""
    P = idx.shape[0]
    S = np.zeros((V, P))
    S[idx, np.arange(P)] = 1.0
    return S


def blur_matrix_bruteforce(coords: np.ndarray) -> np.ndarray:
    """B-bar built by comparing every pair of vertex coordinates: 10 on the
    diagonal (2 per dimension), 1 where two vertices differ by exactly one unit
    in exactly one of the five dimensions, 0 elsewhere."""
    V = coords.shape[0]
    diff = np.abs(coords[:, None, :] - coords[None, :, :])
    unit_step = (diff.sum(axis=2) == 1) & (diff.max(axis=2) == 1)
    B = unit_step.astype(np.float64)
    B[np.arange(V), np.arange(V)] = 2.0 * coords.shape[1]
    return B


def w_hat(S: np.ndarray, m: np.ndarray, n: np.ndarray, B: np.ndarray) -> np.ndarray:
    """W-hat = S^T D_m^-1 D_n B D_n D_m^-1 S (Eq. equiv)."""
    r = n / m
    return S.T @ (r[:, None] * B * r[None, :]) @ S


def pixel_loss(x: np.ndarray, t: np.ndarray, c: np.ndarray, W: np.ndarray, lam: float) -> float:
    """lam/2 sum_ij W_ij (x_i - x_j)^2 + sum_i c_i (x_i - t_i)^2 (Eq. pixel_loss)."""
    d = x[:, None] - x[None, :]
    return 0.5 * lam * float(np.sum(W * d * d)) + float(np.sum(c * (x - t) ** 2))


def pixel_loss_hessian(W: np.ndarray, c: np.ndarray, lam: float) -> np.ndarray:
    """Hessian of pixel_loss in x: 2 lam (diag(row+col sums)/2 - (W + W^T)/2) + 2 diag(c)."""
    L = np.diag(W.sum(axis=1) + W.sum(axis=0)) - W - W.T
    return lam * L + 2.0 * np.diag(c)


def a_literal(m: np.ndarray, n: np.ndarray, B: np.ndarray, sc: np.ndarray, lam: float) -> np.ndarray:
    """A = lam (D_m - D_n B D_n) + diag(S c), dense, exactly as printed (Eq. quad_min)."""
    return lam * (np.diag(m) - n[:, None] * B * n[None, :]) + np.diag(sc)


def solve_dense(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Minimum-norm least-squares solution of A y = b (exact for invertible A)."""
    return np.linalg.lstsq(A, b, rcond=None)[0]


# ----------------------------------------------------------------------------
# Bilateral pyramid (supplement Section 2) as explicit matrices
# ----------------------------------------------------------------------------

def pyramid_splat_matrices(coords: np.ndarray) -> list:
    """[S_0, S_1, ..., S_{K-1}]: S_k maps level-k vertices to level k+1, where
    level k+1's vertices are the distinct coordinates of level k halved (floor),
    until a single vertex remains.  Built by brute force: every level-k vertex
    is compared with every distinct halved coordinate.  The order of a level's
    vertices is that of Python's sorted tuples, unrelated to any other code."""
    level = [tuple(int(x) for x in c) for c in coords]
    mats = []
    while len(level) > 1:
        halves = [tuple(x >> 1 for x in c) for c in level]
        nxt = sorted(set(halves))
        S = np.zeros((len(nxt), len(level)))
        for j, h in enumerate(halves):
            for i, u in enumerate(nxt):
                if u == h:
                    S[i, j] = 1.0
        mats.append(S)
        level = nxt
    return mats


def pyramid_lift_matrices(coords: np.ndarray) -> list:
    """[M_0 = I, M_1 = S_0, M_2 = S_1 S_0, ...]: block k of the stacked P."""
    V = coords.shape[0]
    out = [np.eye(V)]
    for S in pyramid_splat_matrices(coords):
        out.append(S @ out[-1])
    return out


def hier_init_dense(coords: np.ndarray, b: np.ndarray, sc: np.ndarray, alpha: float,
                    beta: float) -> np.ndarray:
    """y_hier = P^T(w o P(b) / P(1)) / P^T(w o P(S c) / P(1)) (Section 4) with
    the stacked P of pyramid_lift_matrices and w = 1 at k = 0, alpha^-(beta+k)
    at k >= 1."""
    Ms = pyramid_lift_matrices(coords)
    ones = np.ones(coords.shape[0])
    num = np.zeros(coords.shape[0])
    den = np.zeros(coords.shape[0])
    for k, M in enumerate(Ms):
        w = 1.0 if k == 0 else float(alpha) ** (-(beta + k))
        cnt = M @ ones
        num += M.T @ (w * (M @ b) / cnt)
        den += M.T @ (w * (M @ sc) / cnt)
    return num / den


def hier_precond_dense(coords: np.ndarray, diag: np.ndarray, alpha: float,
                       beta: float) -> np.ndarray:
    """M_hier^-1 = P^T D P as a dense V x V matrix (Section 4, Eq. hier_precond),
    D = diag(w o P(1) / P(diag A)), with a zero weight where P(diag A) = 0."""
    Ms = pyramid_lift_matrices(coords)
    ones = np.ones(coords.shape[0])
    out = np.zeros((coords.shape[0], coords.shape[0]))
    for k, M in enumerate(Ms):
        w = 1.0 if k == 0 else float(alpha) ** (-(beta + k))
        pd = M @ diag
        scale = np.where(pd > 0, w * (M @ ones) / np.where(pd > 0, pd, 1.0), 0.0)
        out += M.T @ (scale[:, None] * M)
    return out
