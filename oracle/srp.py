"""Sequential random pivoting (SRP, Algorithm 1 of section 3) in plain FP64.
Test infrastructure only.

What is computed (the paper's n x d data matrix is m x n here): skeleton rows
chosen one at a time, each drawn from the squared-norm distribution of the
current residual X (I - Q Q^T).  The drawn row's residual direction q (the
row minus its projection on span(Q), normalised) joins the orthonormal basis;
the factor L gains the column X q, zero on the rows of earlier skeletons; and
every residual squared row norm drops by the square of that row's entry of
X q (Pythagoras over the orthonormal basis).  The loop ends once the
residual's squared Frobenius norm is at most eps^2 ||X||_F^2.

Used as an independent special case of Algorithm 2: with b = 1 the robust
filter keeps the single sampled row (tau_b = 1/1 and tail_1 >= tail_1), so
RBRP with b = 1 and SRP select the same skeletons from the same random stream.

Readings: the loop condition printed in Algorithm 1 compares with "<"; it is
read as ">" as in Algorithm 2 (continue while the residual is above the
tolerance).  The single draw per step uses the same fixed-point draw as the
block sampler with b = 1 (its first candidate), and the direction is
projected twice as in the block form.
"""

import numpy as np

from .sampler import sample_block


def srp(X, eps, seed, k_max=None, ident=0):
    X = np.asarray(X, dtype=np.float64)
    m, n = X.shape
    if k_max is None or k_max <= 0:
        k_max = min(m, n)
    tau = eps * eps
    d = np.einsum("ij,ij->i", X, X)
    D0 = float(d.sum())
    S = []
    in_S = np.zeros(m, dtype=bool)
    basis = []            # orthonormal residual directions, one per skeleton
    columns = []          # the columns of L
    t = 0
    while D0 > 0 and d.sum() > tau * D0 and len(S) < k_max:
        t += 1
        drawn = sample_block(d, in_S, 1, seed, t, ident)
        if not drawn:
            break
        s = drawn[0]
        # the drawn row's residual direction: project out span(Q) twice
        r = X[s, :].copy()
        for _ in range(2):
            for q in basis:
                r -= q * (q @ r)
        nr = np.linalg.norm(r)
        if nr == 0.0:
            break
        q = r / nr
        col = X @ q                    # = residual @ q, since q is orthogonal to span(Q)
        col[in_S] = 0.0
        S.append(s)
        in_S[s] = True
        columns.append(col)
        d = d - col * col
        d[in_S] = 0.0
        d = np.maximum(d, 0.0)
        basis.append(q)
    L = np.column_stack(columns) if columns else np.zeros((m, 0))
    return S, L, d, D0
