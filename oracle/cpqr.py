"""Column-pivoted QR of a sampled block and robust blockwise filtering
(Alg. 2, local CPQR and truncation steps; Remark 4.2).  Test infrastructure
only.

The block V (n x b) holds the residuals of the b sampled rows as columns.
Algorithm 2 factors V(:, pi_V) = Q_V R_V with greedy column pivoting (the
greedy squared-norm pivoting of eq. qr_update, applied to the columns of V)
and keeps the first b' columns, where b' is the largest i with
||R_V(i:b, i:b)||_F^2 >= tau_b ||R_V||_F^2.

Readings used here
------------------
* Householder reflections (the paper notes QR updates are carried out by
  Householder reflection in practice, in the footnote to eq. qr_update).
* The pivot at step p is the remaining column with the largest squared norm of
  its trailing part, recomputed from the current matrix at every step (no
  norm downdating).  Exactly equal norms go to the column that came first in
  the sampled order (lowest original position).
* The threshold comparison carries a relative slack of 4 b u (u = 2^-53):
  tail_i >= tau_b * tail_1 * (1 - 4 b u).  The paper's own toy case of
  orthogonal equal-norm columns (rationale for Conjecture 4.4) sits exactly on
  the threshold and must give b' = b.
* If b > n, R_V has n rows and the tails past row n are zero.
"""

import numpy as np

U64 = 2.0 ** -53


def cpqr(V):
    """Householder QR with column pivoting.

    Returns (piv, R, Q): piv is the column order (indices into V's columns),
    R is min(n, b) x b upper trapezoidal, Q is n x min(n, b) with orthonormal
    columns, and V[:, piv] = Q @ R up to rounding.
    """
    A = np.array(V, dtype=np.float64, copy=True)
    n, b = A.shape
    r = min(n, b)
    piv = np.arange(b)
    vs = []
    for p in range(r):
        norms2 = np.einsum("ij,ij->j", A[p:, p:], A[p:, p:])
        best = norms2.max()
        ties = np.flatnonzero(norms2 == best)
        j = p + int(ties[np.argmin(piv[p + ties])])
        if j != p:
            A[:, [p, j]] = A[:, [j, p]]
            piv[[p, j]] = piv[[j, p]]
        x = A[p:, p].copy()
        nx = np.linalg.norm(x)
        if nx == 0.0:
            vs.append(None)
            continue
        alpha = -nx if x[0] >= 0 else nx
        v = x
        v[0] -= alpha
        vv = v @ v
        if vv == 0.0:
            vs.append(None)
            continue
        A[p:, p:] -= np.outer(v, (2.0 / vv) * (v @ A[p:, p:]))
        A[p + 1:, p] = 0.0
        vs.append(v)
    R = np.triu(A[:r, :])
    Q = np.eye(n, r)
    for p in range(r - 1, -1, -1):
        v = vs[p]
        if v is None:
            continue
        Q[p:, :] -= np.outer(v, (2.0 / (v @ v)) * (v @ Q[p:, :]))
    return piv, R, Q


def tails_from_r(R, b):
    """tail_i = ||R(i:b, i:b)||_F^2 for i = 1..b (index 0..b-1 here)."""
    r = R.shape[0]
    tails = np.zeros(b)
    for i in range(min(r, b)):
        tails[i] = float(np.sum(R[i:, i:] ** 2))
    return tails


def truncation_rank(tails, tau_b, b):
    """b' = max{i : tail_i >= tau_b * tail_1} (Alg. 2; Remark 4.2)."""
    thr = tau_b * tails[0] * (1.0 - 4.0 * b * U64)
    ok = np.flatnonzero(tails >= thr)
    return int(ok.max()) + 1 if ok.size else 1


def filter_block(V, tau_b):
    """Local CPQR + truncation.  Returns (piv, R, Q, tails, b')."""
    b = V.shape[1]
    piv, R, Q = cpqr(V)
    tails = tails_from_r(R, b)
    bp = truncation_rank(tails, tau_b, b)
    bp = min(bp, R.shape[0])
    return piv, R, Q, tails, bp
