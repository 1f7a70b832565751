"""CPU FP64 oracle for robust blockwise random pivoting (RBRP) interpolative
decompositions -- TEST INFRASTRUCTURE ONLY.

This package is the parity reference for the GPU library.  It is a plain,
slow, obviously-correct restatement of the paper's method (Dong, Chen,
Martinsson, Pearce, "Robust blockwise random pivoting: fast and accurate
adaptive interpolative decomposition", arXiv:2309.16002) in NumPy/FP64:

* ``philox``   -- Philox4x64-10 counter-based generator (Salmon et al., SC'11).
* ``sampler``  -- squared-norm sampling without replacement from the residual
                  norms (Alg. 2, sampling step; eq. squared_norm_distribution)
                  through an exact fixed-point integer CDF.
* ``cpqr``     -- column-pivoted Householder QR of a sampled block and the
                  robust blockwise truncation (Alg. 2 local CPQR; Remark 4.2).
* ``rbrp``     -- Algorithm 2 (RBRP), literal form (d downdated from
                  L-hat = X Q'), explicit-deflation form (R <- R - (R Q') Q'^T),
                  and the greedy (RBGP, Remark 4.3) selection variant.
* ``srp``      -- Algorithm 1 (sequential random pivoting), used as an
                  independent special case (RBRP with b = 1).
* ``sketchy``  -- sketchy pivoting with LU and partial pivoting on the sketch
                  Y = X Omega (SkLUPP) and the oversampled sketchy
                  interpolation matrix (OSID, Algorithm 4).
* ``interp``   -- interpolation matrix: W = X X_S^+ (eq. stable_id),
                  Algorithm 3 (W from L), and Remark 5.2's truncated-SVD
                  pseudo-inverse of L_1.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it, and it
shares no code with the GPU library; the only common dependency is the seeded
input generators in ``workloads``, which contain none of the method's
arithmetic.

Every function cites the passage of the paper it follows (section, equation,
algorithm, remark).  Readings of passages that are silent or ambiguous are
stated at the function that implements them; all of them are collected in the
project's design document.
"""

from .philox import philox4x64_10, philox_word0
from .sampler import fixed_point_weights, sample_block
from .cpqr import cpqr, truncation_rank, tails_from_r
from .rbrp import rbrp, RBRPResult
from .srp import srp
from .interp import w_lstsq, w_from_l, w_svd_pinv, relative_id_error
from .trim import trim_rank, projection_error_sq
from .sketchy import sketch, lupp_pivots, osid, sketchy_id

__all__ = [
    "philox4x64_10", "philox_word0", "fixed_point_weights", "sample_block",
    "cpqr", "truncation_rank", "tails_from_r", "rbrp", "RBRPResult", "srp",
    "w_lstsq", "w_from_l", "w_svd_pinv", "relative_id_error", "trim_rank", "projection_error_sq",
    "sketch", "lupp_pivots", "osid", "sketchy_id",
]
