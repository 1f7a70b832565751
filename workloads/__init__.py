"""Seeded synthetic input generators for RBRP interpolative decompositions.

This module produces input matrices only.  It contains none of the method's
arithmetic and is the one piece of code shared by the CPU oracle's tests, the
GPU library's tests and the benchmark.  Every generator is deterministic in
its seed (NumPy PCG64) and runs on the CPU.

Workloads (the paper's n x d data matrix is written m x n here):

* ``svd_matrix``      X = U diag(s) V^T with Haar-distributed orthonormal U, V
                      (the construction of the paper's Gaussian-exp matrix,
                      Section 6.1); ``geometric_spectrum`` (s_i = q^i) and
                      ``power_spectrum`` (s_i = i^-p) give the decays used.
* ``adversarial_gmm`` rows from a Gaussian mixture whose means have distinct
                      norms, in the style of Example 4.1, with power-law
                      cluster sizes, a low-dimensional subspace and
                      near-duplicate rows.
* ``gmm_example41``   Example 4.1 exactly: means 10 j e_j, identity covariance,
                      equal cluster sizes.
* ``example23``       Example 2.3: scaled canonical basis vectors repeated.
* ``kernel_blocks``   Gaussian-kernel blocks exp(-|x-y|^2/h^2) between
                      separated 3-D point clusters (off-diagonal blocks of a
                      hierarchical matrix, cf. the paper's fast-direct-solver
                      remark).
* ``random_features`` cos(x Omega + c) for x from a GMM in R^64.
* ``exact_rank``      a matrix of exact rank r.
* ``gaussian_exp``    the Gaussian-exp matrix of section 6: Haar factors and a
                      spectrum flat for 100 values, then 0.8^(i-100) floored
                      at 1e-5.
"""

from .generators import (
    haar, svd_matrix, geometric_spectrum, power_spectrum, adversarial_gmm,
    gmm_example41, example23, kernel_blocks, random_features, exact_rank,
    gaussian_exp, gaussian_exp_spectrum, config_matrix, CONFIGS,
)

__all__ = [
    "haar", "svd_matrix", "geometric_spectrum", "power_spectrum",
    "adversarial_gmm", "gmm_example41", "example23", "kernel_blocks",
    "random_features", "exact_rank", "gaussian_exp", "gaussian_exp_spectrum",
    "config_matrix", "CONFIGS",
]
