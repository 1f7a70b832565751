"""Interpolation matrix construction (Section 5).  Test infrastructure only.

* ``w_lstsq``  -- the optimal interpolation matrix W = X X_S^+, the
  least-squares solution of min_W ||X - W X_S||_F (eq. stable_id), computed by
  LAPACK least squares in FP64.  This is the plain definition of the result.
* ``w_from_l`` -- Algorithm 3: with L_1 = L(S,:) (k x k) and the remaining
  rows L_2, W(S,:) = I and W(rest,:) = L_2 L_1^{-1}.  Prop. 5.1 shows this
  equals X X_S^+ in exact arithmetic.  L_1 is lower triangular (rows of earlier
  skeletons are zero in later blocks of L), so L_2 L_1^{-1} is a triangular
  solve, as the paper notes after Prop. 5.1.
* ``w_svd_pinv`` -- the stable evaluation of Remark 5.2: W(S,:) = I and
  W(rest,:) = L_2 L_1^+ with L_1^+ the pseudo-inverse of the truncated SVD of
  L_1, singular values below ``clip`` dropped with their singular vectors.
  Reading: the tolerance is relative to the largest singular value of L_1
  (the paper says "below a given tolerance, e.g. 10^-12" without a scale).
  Without truncation this is Alg. 3's W.
* ``relative_id_error`` -- ||X - W X_S||_F / ||X||_F (errors are normalised by
  ||X||_F in the paper's experiments).
"""

import numpy as np
import scipy.linalg


def w_lstsq(X, S):
    X = np.asarray(X, dtype=np.float64)
    S = list(S)
    if not S:
        return np.zeros((X.shape[0], 0))
    XS = X[S, :]                                  # k x n
    # min_W ||X - W XS||_F  <=>  XS^T W^T = X^T in the least-squares sense
    Wt, *_ = np.linalg.lstsq(XS.T, X.T, rcond=None)
    return Wt.T


def w_from_l(L, S):
    L = np.asarray(L, dtype=np.float64)
    S = list(S)
    m, k = L.shape
    W = np.zeros((m, k))
    if k == 0:
        return W
    L1 = np.tril(L[S, :])                         # k x k, lower triangular
    rest = np.ones(m, dtype=bool)
    rest[S] = False
    # W2 L1 = L2  <=>  L1^T W2^T = L2^T  (upper-triangular solve)
    W2t = scipy.linalg.solve_triangular(L1.T, L[rest, :].T, lower=False)
    W[rest, :] = W2t.T
    W[S, :] = np.eye(k)
    return W


def w_svd_pinv(L, S, clip=1e-12):
    """Remark 5.2: W = L L_1^+ through the truncated SVD of L_1 = L(S,:)
    (lower triangular), with W(S,:) = I.  Returns (W, number of singular
    values kept)."""
    L = np.asarray(L, dtype=np.float64)
    S = list(S)
    m, k = L.shape
    W = np.zeros((m, k))
    if k == 0:
        return W, 0
    L1 = np.tril(L[S, :])
    U, sv, Vt = np.linalg.svd(L1)
    keep = sv >= clip * sv[0]
    r = int(np.count_nonzero(keep))
    # L_1^+ = V_r diag(1 / s_r) U_r^T
    P = (Vt[keep].T / sv[keep]) @ U[:, keep].T
    W = L @ P
    W[S, :] = np.eye(k)
    return W, r


def relative_id_error(X, W, S):
    X = np.asarray(X, dtype=np.float64)
    nx = np.linalg.norm(X)
    if nx == 0.0:
        return 0.0
    S = list(S)
    if not S:
        return 1.0
    return float(np.linalg.norm(X - W @ X[S, :]) / nx)
