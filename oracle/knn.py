"""Stencil membership (Sec. 4): node x_1 plus its n-1 nearest neighbours.

Distances are Euclidean in R^3 (straight-line, not along the surface).  The
stencil size n counts the centre, which always takes slot 0; the other n-1
nodes are ascending by (squared distance, node index).  The squared distance
is formed as ((dx*dx + dy*dy) + dz*dz) in FP64 with no fused multiply-add, so
that the order is exactly reproducible.

Parity pin: brute force on tiny inputs and exact-tie lattices (tests).
"""
from __future__ import annotations

import numpy as np

__all__ = ["sqdist_rows", "knn_bruteforce", "knn"]


def sqdist_rows(X: np.ndarray, i: int, cand: np.ndarray) -> np.ndarray:
    """((dx*dx + dy*dy) + dz*dz) from node i to the candidate nodes."""
    d = X[cand] - X[i]
    dx, dy, dz = d[:, 0], d[:, 1], d[:, 2]
    return (dx * dx + dy * dy) + dz * dz


def _order(i: int, d2: np.ndarray, cand: np.ndarray, n: int) -> np.ndarray:
    # centre first, then ascending by (d2, index); lexsort sorts by the last key first
    keep = cand != i
    c, d = cand[keep], d2[keep]
    o = np.lexsort((c, d))
    return np.concatenate([[i], c[o[:n - 1]]])


def knn_bruteforce(X: np.ndarray, n: int) -> np.ndarray:
    """All-pairs kNN, O(N^2): idx[i, 0] == i, then ascending (d^2, index)."""
    N = len(X)
    if n > N:
        raise ValueError("stencil size exceeds node count")
    out = np.empty((N, n), dtype=np.int64)
    allidx = np.arange(N)
    for i in range(N):
        out[i] = _order(i, sqdist_rows(X, i, allidx), allidx, n)
    return out


def knn(X: np.ndarray, n: int, rows=None) -> np.ndarray:
    """kNN for the given rows (default: all), exact in (d^2, index) order.

    A k-d tree proposes candidates; every candidate set is re-ranked by the
    exact FP64 squared distance and index, and the query is widened until the
    n-th distance is strictly below the largest candidate distance, so ties
    at the boundary are resolved by index exactly as brute force would.
    """
    from scipy.spatial import cKDTree

    N = len(X)
    if n > N:
        raise ValueError("stencil size exceeds node count")
    rows = np.arange(N) if rows is None else np.asarray(rows)
    if N <= 4096:
        out = np.empty((len(rows), n), dtype=np.int64)
        allidx = np.arange(N)
        for t, i in enumerate(rows):
            out[t] = _order(i, sqdist_rows(X, i, allidx), allidx, n)
        return out
    tree = cKDTree(X)
    out = np.empty((len(rows), n), dtype=np.int64)
    k = min(N, n + 16)
    _, cand = tree.query(X[rows], k=k)
    for t, i in enumerate(rows):
        c = np.asarray(cand[t])
        kk = k
        while True:
            c = c[c != i]
            d2 = sqdist_rows(X, i, c)
            o = np.lexsort((c, d2))
            if kk >= N or d2[o[n - 2]] < d2.max() * (1.0 - 1e-12):
                out[t] = np.concatenate([[i], c[o[:n - 1]]])
                break
            kk = min(N, 2 * kk)
            _, c = tree.query(X[i], k=kk)
            c = np.asarray(c)
    return out
