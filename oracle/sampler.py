"""Squared-norm sampling without replacement (Alg. 2, sampling step), made
exact with a fixed-point integer CDF.  Test infrastructure only.

What the paper fixes
--------------------
Block t of Algorithm 2 draws b indices "without replacement" from the
residual squared-norm distribution d^(t-1) / ||d^(t-1)||_1 (Alg. 2; the
squared-norm distribution is eq. squared_norm_distribution applied to the
residual, as in Alg. 1).  The paper names no sampling scheme, no probability
representation and no generator.

Readings used here (shared by both implementations so that skeletons are
bit-exact when both see the same d and the same random stream)
--------------------------------------------------------------------------
* Probabilities as integers.  Let dmax = max_i max(d_i, 0) over rows not yet
  selected, written dmax = f * 2^e with f in [0.5, 1) (frexp).  With
  s = 62 - e - ceil(log2 m), every weight is w_i = floor(max(d_i, 0) * 2^s)
  (an exact scaling by a power of two), and w_i = 0 for selected rows.  Then
  sum_i w_i < 2^62, and the inclusive prefix C of w is exact in uint64.
* One draw.  A 64-bit word x gives target = floor(x * W / 2^64) with
  W = C[m-1] (exact 128-bit product); the drawn index is the smallest i with
  C_i > target.  Index i is drawn with probability w_i / W (to within 2^-64).
* Without replacement = successive sampling.  Candidates j = 0, 1, 2, ... are
  drawn from the fixed CDF of the block and a candidate is accepted when its
  index has not been accepted before; this stops at b accepted indices.
  Rejecting repeats makes every accepted index a draw from the weights of the
  rows not yet drawn, which is successive sampling.
* Termination.  If at most b rows have positive weight, all of them are taken
  in increasing index order.  If J_max = 32 b candidates pass before b are
  accepted, the remaining draws switch to "removal" form: the weights of the
  accepted rows are set to zero, the CDF is rebuilt, and each further counter
  j >= J_max yields one accepted index.  The distribution is unchanged.
"""

import math

import numpy as np

from .philox import philox_word0

REJECTION_FACTOR = 32  # J_max = REJECTION_FACTOR * b


def _ceil_log2(m):
    return 0 if m <= 1 else (int(m) - 1).bit_length()


def fixed_point_weights(d, excluded=None):
    """Integer weights w (uint64) and the scale exponent s.

    d        : FP64 residual squared row norms (Alg. 2, d^(t-1)).
    excluded : boolean mask of rows already in S (weight forced to zero).
    """
    d = np.asarray(d, dtype=np.float64)
    m = d.shape[0]
    dpos = np.maximum(d, 0.0)
    if excluded is not None:
        dpos = np.where(np.asarray(excluded, dtype=bool), 0.0, dpos)
    dmax = float(dpos.max()) if m else 0.0
    if dmax <= 0.0:
        return np.zeros(m, dtype=np.uint64), 0
    _, e = math.frexp(dmax)
    s = 62 - e - _ceil_log2(m)
    w = np.floor(np.ldexp(dpos, s)).astype(np.uint64)
    return w, s


def _draw(C, x):
    """Index of the smallest inclusive prefix value above the target."""
    W = int(C[-1])
    target = (int(x) * W) >> 64
    return int(np.searchsorted(C, np.uint64(target), side="right"))


def sample_block(d, excluded, b, seed, t, ident=0):
    """Draw one block S_t of at most ``b`` distinct row indices (Alg. 2).

    Returns the indices in acceptance order (a Python list of ints).
    """
    w, _ = fixed_point_weights(d, excluded)
    positive = np.flatnonzero(w)
    if positive.size <= b:
        return [int(i) for i in positive]
    C = np.cumsum(w, dtype=np.uint64)
    accepted = []
    seen = set()
    j = 0
    j_max = REJECTION_FACTOR * b
    while len(accepted) < b and j < j_max:
        idx = _draw(C, philox_word0(j, t, ident, seed))
        if idx not in seen:
            seen.add(idx)
            accepted.append(idx)
        j += 1
    while len(accepted) < b:
        w_left = w.copy()
        w_left[accepted] = 0
        C_left = np.cumsum(w_left, dtype=np.uint64)
        idx = _draw(C_left, philox_word0(j, t, ident, seed))
        accepted.append(idx)
        j += 1
    return accepted


def top_b(d, excluded, b):
    """Greedy selection of Remark 4.3 (RBGP): the b largest residual norms.

    Rows with d_i <= 0 are never chosen; equal values go to the lower index.
    """
    d = np.asarray(d, dtype=np.float64).copy()
    if excluded is not None:
        d[np.asarray(excluded, dtype=bool)] = 0.0
    cand = np.flatnonzero(d > 0.0)
    order = sorted(cand.tolist(), key=lambda i: (-d[i], i))
    return order[:b]
