"""Sketchy pivoting with LU and partial pivoting (SkLUPP) and the oversampled
sketchy interpolation matrix (OSID, Algorithm 4 of section 5) in plain FP64.
Test infrastructure only.

What is computed (the paper's n x d data matrix is m x n here), following
the two stages of sketchy pivoting described in section 3 and Algorithm 4:

* the sketch Y = X Omega (m x l) with a caller-supplied embedding Omega
  (n x l; the paper draws it Gaussian);
* skeletons: the first k pivot rows of Gaussian elimination with partial
  pivoting on Y -- at step j the active row with the largest |entry| in
  column j of the current Schur complement (ties to the lowest row index),
  which is then eliminated from the other active rows.  Only columns
  0 .. k-1 of Y decide the first k pivots;
* OSID: with Y_S = Y(S,:) (k x l) and its thin QR Y_S^T = Q R,
  W = (Y Q) R^{-T} = Y Y_S^+, W(S,:) = I.

Readings (where the paper is silent): a column whose active entries are all
zero pivots on its lowest active row and eliminates nothing; k <= l, k <= m.
"""

import numpy as np
import scipy.linalg


def sketch(X, Omega):
    return np.asarray(X, dtype=np.float64) @ np.asarray(Omega, dtype=np.float64)


def lupp_pivots(Y, k):
    """First k pivot rows of partial-pivoting elimination on Y(:, 0:k)."""
    Z = np.array(Y[:, :k], dtype=np.float64)
    m = Z.shape[0]
    active = np.ones(m, dtype=bool)
    piv = []
    for j in range(k):
        col = np.where(active, np.abs(Z[:, j]), -1.0)
        p = int(np.argmax(col))          # first maximum: lowest index on ties
        piv.append(p)
        active[p] = False
        if Z[p, j] != 0.0:
            mult = np.where(active, Z[:, j] / Z[p, j], 0.0)
            Z[:, j + 1:] -= np.outer(mult, Z[p, j + 1:])
    return piv


def osid(Y, S):
    """Algorithm 4: W = (Y Q) R^{-T} with Y(S,:)^T = Q R; W(S,:) = I."""
    Y = np.asarray(Y, dtype=np.float64)
    S = list(S)
    k = len(S)
    Q, R = np.linalg.qr(Y[S].T)                   # l x k, k x k
    # W R^T = Y Q  <=>  R W^T = (Y Q)^T
    W = scipy.linalg.solve_triangular(R, (Y @ Q).T, lower=False).T
    W[S, :] = np.eye(k)
    return W


def sketchy_id(X, Omega, k):
    """SkLUPP skeletons and the OSID interpolation matrix; returns (S, W, Y)."""
    Y = sketch(X, Omega)
    S = lupp_pivots(Y, k)
    return S, osid(Y, S), Y
