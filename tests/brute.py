"""Independent brute-force and closed-form helpers for pinning the oracle.

Nothing here calls the oracle or the GPU library.  Distances come from
scipy's all-pairs shortest paths (a library routine), layouts are handled as
dense numpy arrays, and every quantity is computed from its definition over
all pairs rather than by the incremental steps the oracle takes.
"""
from __future__ import annotations

import numpy as np


def apsp(g) -> np.ndarray:
    """All-pairs hop distances via scipy.sparse.csgraph (int64, n x n)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path

    a = sp.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    d = shortest_path(a, method="D", unweighted=True, directed=False)
    if np.isinf(d).any():
        raise ValueError("disconnected")
    return d.astype(np.int64)


def maxmin_brute(D: np.ndarray, k: int, first: int) -> list[int]:
    """Max/min sp sampling over the full distance matrix."""
    piv = [first]
    while len(piv) < k:
        m = D[piv].min(axis=0)
        piv.append(int(np.argmax(m)))  # argmax returns the first (lowest id) maximum
    return piv


def weights_brute(D: np.ndarray, pivots, region) -> np.ndarray:
    """w'_{ip} = s / d_ip^2, s = |{j in R(p): d_jp <= d_ip / 2}| over the reals,
    zero where d_ip < 2.  Returns an n x k matrix (node, pivot rank)."""
    n = D.shape[0]
    k = len(pivots)
    W = np.zeros((n, k))
    for t, p in enumerate(pivots):
        members = np.flatnonzero(np.asarray(region) == t)
        djp = D[p, members].astype(np.float64)
        for i in range(n):
            d = float(D[i, p])
            if d < 2:
                continue
            s = int(np.count_nonzero(djp <= d / 2.0))
            W[i, t] = s / (d * d)
    return W


def full_stress(D: np.ndarray, x: np.ndarray) -> float:
    """Eq. 1 over all pairs i < j with w = d^-2."""
    n = D.shape[0]
    iu = np.triu_indices(n, 1)
    diff = x[:, None, :] - x[None, :, :]
    r = np.sqrt((diff ** 2).sum(-1))[iu]
    d = D[iu].astype(np.float64)
    return float(((r - d) ** 2 / d ** 2).sum())


def localized_full_step(D: np.ndarray, x: np.ndarray) -> np.ndarray:
    """One Jacobi sweep of the localized full-stress update (the equation
    before Eq. 5 in Section 3): all j != i, w_ij = d_ij^-2."""
    n = D.shape[0]
    out = np.empty_like(x)
    for i in range(n):
        j = np.arange(n) != i
        d = D[i, j].astype(np.float64)
        w = 1.0 / d ** 2
        diff = x[i] - x[j]
        r = np.sqrt((diff ** 2).sum(-1))
        with np.errstate(invalid="ignore", divide="ignore"):
            vote = x[j] + np.where(r[:, None] > 0, d[:, None] * diff / r[:, None], 0.0)
        out[i] = (w[:, None] * vote).sum(0) / w.sum()
    return out


def procrustes_align(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Rigidly move X (rotation or reflection plus translation, no scaling)
    onto Y in the least-squares sense; returns the moved X."""
    mx, my = X.mean(0), Y.mean(0)
    A, B = X - mx, Y - my
    U, _, Vt = np.linalg.svd(A.T @ B)
    R = U @ Vt
    return A @ R + my


def coord_error(x: np.ndarray, ref: np.ndarray, align: bool = False) -> float:
    """max_i ||x_i - ref_i|| / RMS radius of ref (after optional alignment)."""
    if align:
        x = procrustes_align(x, ref)
    rad = np.sqrt(((ref - ref.mean(0)) ** 2).sum(1).mean())
    return float(np.sqrt(((x - ref) ** 2).sum(1)).max() / rad)
