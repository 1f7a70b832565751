"""Rank trimming after Algorithm 2.  Test infrastructure only.

Algorithm 2 applies its stopping rule only between blocks, so the last block
can add up to b' - 1 skeletons beyond what the tolerance needs (the paper
accepts this overshoot when it discusses the block size).  The trimmed rank
is the shortest prefix S(1:j) of the selection whose skeletonization error
meets the tolerance:

    k' = min{ j : ||X - X Q_j Q_j^T||_F^2 <= eps^2 ||X||_F^2 },

with Q_j the first j columns of the orthonormal basis Algorithm 2 builds.
Each block's basis is the orthonormalised projection of its kept rows, in
their pivoted order, so span(Q_j) = span(X(S(1:j),:)^T), and by Prop. 5.1
the quantity above is the error of the interpolative decomposition on
S(1:j).  If no prefix meets it (possible only through rounding at the last
one), k' = k.

W for the prefix is Algorithm 3 applied to the leading k' columns of L:
L_1 = L(S,:) is lower triangular, so its leading k' x k' block is the L_1 of
the prefix.
"""

import numpy as np


def projection_error_sq(X, Qt, j):
    """||X - X Q_j Q_j^T||_F^2 with Q_j^T the first j rows of Qt."""
    X = np.asarray(X, dtype=np.float64)
    if j == 0:
        return float(np.sum(X * X))
    Qj = np.asarray(Qt, dtype=np.float64)[:j, :].T          # n x j
    E = X - (X @ Qj) @ Qj.T
    return float(np.sum(E * E))


def trim_rank(X, res, eps):
    """Smallest j with projection_error_sq(X, res.Qt, j) <= eps^2 ||X||_F^2.

    Returns (k', error_sq) for the RBRPResult ``res`` of Algorithm 2 on X.
    Every prefix j = 0, 1, ..., k is tried in order (the literal definition).
    """
    X = np.asarray(X, dtype=np.float64)
    D0 = float(np.sum(X * X))
    thr = eps * eps * D0
    e = D0
    for j in range(0, res.k + 1):
        e = projection_error_sq(X, res.Qt, j)
        if e <= thr:
            return j, e
    return res.k, e
