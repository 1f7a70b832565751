"""Algorithm 1 -- sequential random pivoting (SRP) -- in plain FP64.
Test infrastructure only.

Used as an independent special case of Algorithm 2: with b = 1 the robust
filter keeps the single sampled row (tau_b = 1/1 and tail_1 >= tail_1), so
RBRP with b = 1 and SRP select the same skeletons from the same random stream.

Per step (Alg. 1), with the paper's n x d matrix written m x n here:
  s_t ~ d / ||d||_1
  v   <- x_{s_t} - Q (Q^T x_{s_t});  Q <- [Q, v / ||v||]
  a   <- X(pi_a,:) v  on the active rows (zero on earlier skeletons)
  L   <- [L, a / sqrt(a(s_t))]
  d_i <- 0 for i in S,  d_i <- d_i - a_i^2 / a(s_t) otherwise

Reading: the loop condition printed in Alg. 1 compares with "<"; it is read
as ">" as in Algorithm 2 (continue while the residual is above tolerance).
The single draw per step uses the same fixed-point draw as the block sampler
with b = 1 (its first candidate), and v is projected twice as in the block
form.
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
    Qcols = []
    Lcols = []
    t = 0
    while D0 > 0 and d.sum() > tau * D0 and len(S) < k_max:
        t += 1
        drawn = sample_block(d, in_S, 1, seed, t, ident)
        if not drawn:
            break
        s = drawn[0]
        v = X[s, :].copy()
        for _ in range(2):
            for q in Qcols:
                v -= q * (q @ v)
        nv = np.linalg.norm(v)
        if nv == 0.0:
            break
        a = X @ v                      # unnormalised v, as in Alg. 1
        a[in_S] = 0.0
        S.append(s)
        in_S[s] = True
        a_s = a[s]                     # equals ||v||^2 = d(s) in exact arithmetic
        Lcols.append(a / np.sqrt(a_s))
        d = d - a * a / a_s
        d[in_S] = 0.0
        d = np.maximum(d, 0.0)
        Qcols.append(v / nv)
    L = np.column_stack(Lcols) if Lcols else np.zeros((m, 0))
    return S, L, d, D0
