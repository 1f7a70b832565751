"""Robust blockwise random pivoting (RBRP, Algorithm 2 of section 4) in plain
FP64.  Test infrastructure only.

What is computed (the paper's n x d data matrix is m x n here): an ordered
set S of skeleton rows of X, grown one block at a time.  A block draws b rows
from the squared-norm distribution of the current residual X (I - Q Q^T)
(section 2.2's distribution, applied to the residual), removes from them the
part the current orthonormal basis Q already spans, and keeps the b' of them
that a column-pivoted QR ranks first, cut where the rest carries less than
tau_b of the block's projected mass (the robust truncation of Remark 4.2).
The kept rows join S, their orthonormal directions Q' join Q, and X Q' (zero
on the rows of earlier skeletons) joins the factor L from which Algorithm 3
forms W.  The loop ends once the residual's squared Frobenius norm is at
most eps^2 ||X||_F^2, or at k_max rows.

The residual row norms d are kept in one of two ways, which give the same
skeletons in exact arithmetic (Q' is orthogonal to Q, so R Q' = X Q'):

* form "A" downdates d by the squared rows of X Q', as the paper describes
  (the timed CPU baseline);
* form "B" stores the residual R = X (I - Q Q^T) and recomputes its row norms
  after each block; this is the form the GPU library implements.

Readings (where the paper is silent or ambiguous)
-------------------------------------------------
* tau = eps^2: ``eps`` is a relative Frobenius tolerance, and the paper's tau
  bounds the relative squared residual ||d||_1 / ||d^(0)||_1.
* The projection is applied twice (classical Gram-Schmidt with one
  re-orthogonalisation), always from the original rows X(S_t,:); the paper
  stresses keeping the basis orthonormal to high precision (Remark 2.1).
* Negative d from rounding is clamped to zero.
* The loop also ends when the sampled block is numerically inside span(Q)
  (||V||_F <= 1e-13 ||X(S_t,:)||_F): no further direction can be resolved in
  FP64.  This only triggers when eps is below the arithmetic's floor.
* tau_b defaults to 1/b for the nominal b; fixed-rank mode keeps it when the
  last block is shortened.
* ``greedy=True`` replaces the sampling by the b largest residual norms
  (RBGP, Remark 4.3).
"""

from dataclasses import dataclass, field

import numpy as np

from .cpqr import filter_block
from .sampler import sample_block, top_b

RANK_GUARD = 1e-13


@dataclass
class RBRPResult:
    S: list                      # skeleton indices in selection order
    k: int
    L: np.ndarray                # m x k
    Qt: np.ndarray               # k x n, orthonormal rows (Q^T)
    d: np.ndarray                # final residual squared row norms
    D0: float
    blocks: list = field(default_factory=list)   # per block: (S_t, b')
    resid_sq: float = 0.0        # ||d||_1 at exit

    @property
    def rho(self):
        """Tracked relative residual sqrt(||d||_1 / ||d^(0)||_1)."""
        return float(np.sqrt(self.resid_sq / self.D0)) if self.D0 > 0 else 0.0


def rbrp(X, eps, b, seed, tau_b=None, k_max=None, form="B", greedy=False,
         fixed_rank=False, ident=0, trace=None):
    """Run Algorithm 2 on X (m x n, FP64).  Returns an RBRPResult.

    ``trace``: a list to which a copy of the residual norms each block
    samples from is appended (no effect on the result)."""
    X = np.asarray(X, dtype=np.float64)
    m, n = X.shape
    if tau_b is None:
        tau_b = 1.0 / b
    if k_max is None or k_max <= 0:
        k_max = min(m, n)
    tau = eps * eps

    d = np.einsum("ij,ij->i", X, X)
    D0 = float(d.sum())
    S = []
    in_S = np.zeros(m, dtype=bool)
    Qt = np.zeros((0, n))
    L = np.zeros((m, 0))
    blocks = []
    if D0 == 0.0:
        return RBRPResult(S, 0, L, Qt, d, D0, blocks, 0.0)
    R = X.copy() if form == "B" else None
    t = 0
    while len(S) < k_max and (fixed_rank or d.sum() > tau * D0):
        t += 1
        b_t = min(b, k_max - len(S))
        if trace is not None:
            trace.append(d.copy())
        if greedy:
            S_t = top_b(d, in_S, b_t)
        else:
            S_t = sample_block(d, in_S, b_t, seed, t, ident)
        if not S_t:
            break
        XS = X[S_t, :]                          # b_t x n
        V = XS.T.copy()                         # n x b_t
        for _ in range(2):
            V -= Qt.T @ (Qt @ V)
        if np.linalg.norm(V) <= RANK_GUARD * np.linalg.norm(XS):
            break
        piv, _, QV, _, bp = filter_block(V, tau_b)
        S_new = [S_t[int(piv[i])] for i in range(bp)]
        Qn = QV[:, :bp]                         # n x b'
        if form == "A":
            Lhat = X @ Qn
            Lhat[in_S, :] = 0.0
            d = d - np.einsum("ij,ij->i", Lhat, Lhat)
        else:
            P = R @ Qn
            R -= P @ Qn.T
            Lhat = P
            Lhat[in_S, :] = 0.0
            d = np.einsum("ij,ij->i", R, R)
        S.extend(S_new)
        in_S[S_new] = True
        d[in_S] = 0.0
        d = np.maximum(d, 0.0)
        Qt = np.vstack([Qt, Qn.T])
        L = np.hstack([L, Lhat])
        blocks.append((list(S_t), bp))
    return RBRPResult(S, len(S), L, Qt, d, D0, blocks, float(d.sum()))
