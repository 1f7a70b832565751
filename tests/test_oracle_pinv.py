"""Pins for the oracle's truncated-SVD interpolation matrix (Remark 5.2),
``w_svd_pinv``: W(S,:) = I, W(rest,:) = L_2 L_1^+ with the singular values
of L_1 below clip * sigma_max dropped.

* Without truncation it is Alg. 3's W (an independent triangular solve) and
  X X_S^+ (least squares), Prop. 5.1.
* A diagonal L_1 has its pseudo-inverse in closed form.
* A lower-triangular L_1 with prescribed singular values (the Cholesky factor
  of U diag(s^2) U^T) is checked against the truncated inverse built from the
  symmetric eigendecomposition of L_1^T L_1 (a different LAPACK route than the
  SVD), and the number of values kept against the prescribed spectrum.
"""

import numpy as np
import pytest

from oracle import rbrp, w_from_l, w_lstsq, w_svd_pinv
from workloads import svd_matrix, geometric_spectrum, haar


def test_without_truncation_equals_alg3_and_lstsq():
    X = svd_matrix(600, 150, geometric_spectrum(150, 0.9), seed=31)
    r = rbrp(X, 1e-3, 16, seed=2)
    W, kept = w_svd_pinv(r.L, r.S, clip=1e-12)
    assert kept == r.k
    W3 = w_from_l(r.L, r.S)
    Wl = w_lstsq(X, r.S)
    assert np.array_equal(W[r.S], np.eye(r.k))
    assert np.linalg.norm(W - W3) <= 1e-10 * np.linalg.norm(W3)
    assert np.linalg.norm(W - Wl) <= 1e-10 * np.linalg.norm(Wl)


def _embed(L1, L2, seed):
    """An m x k factor whose rows S are L1 (rows placed at random positions)."""
    rng = np.random.default_rng(seed)
    k = L1.shape[0]
    m = k + L2.shape[0]
    perm = rng.permutation(m)
    S = [int(i) for i in perm[:k]]
    rest = perm[k:]
    L = np.zeros((m, k))
    L[S] = L1
    L[rest] = L2
    return L, S, rest


def test_diagonal_factor_closed_form():
    rng = np.random.default_rng(5)
    # 2e-12 lies between the absolute 1e-12 and the relative 1e-12 * 3: the
    # relative reading drops it
    d = np.array([3.0, -1.0, 2e-12, 0.5, -4e-14, 1e-9])
    L1 = np.diag(d)
    L2 = rng.standard_normal((40, d.size))
    L, S, rest = _embed(L1, L2, 6)
    W, kept = w_svd_pinv(L, S, clip=1e-12)
    # relative clip: 1e-12 * 3 = 3e-12 drops 2e-12 and 4e-14
    keep = np.abs(d) >= 1e-12 * np.abs(d).max()
    assert kept == int(keep.sum()) == 4
    expect = L2 * np.where(keep, 1.0 / np.where(keep, d, 1.0), 0.0)
    assert np.allclose(W[rest], expect, rtol=1e-14, atol=0.0)
    assert np.array_equal(W[S], np.eye(d.size))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_prescribed_spectrum_against_eigendecomposition(seed):
    rng = np.random.default_rng(100 + seed)
    k = 30
    # singular values 1 ... 1e-6, the clip 1e-3 between the 15th and 16th
    s = np.concatenate([np.logspace(0, -2.5, 15), np.logspace(-3.6, -6, 15)])
    U = haar(rng, k, k)
    L1 = np.linalg.cholesky((U * s ** 2) @ U.T)      # lower triangular, sigma(L1) = s
    assert np.allclose(np.linalg.svd(L1, compute_uv=False), np.sort(s)[::-1], rtol=1e-6)
    L2 = rng.standard_normal((200, k))
    L, S, rest = _embed(L1, L2, seed)
    W, kept = w_svd_pinv(L, S, clip=1e-3)
    assert kept == 15
    # truncated inverse from L1^T L1 = V diag(s^2) V^T: L1^+ = V_r diag(s_r^-2) V_r^T L1^T
    lam, V = np.linalg.eigh(L1.T @ L1)
    big = lam >= (1e-3 * s.max()) ** 2
    assert int(big.sum()) == 15
    P = (V[:, big] / lam[big]) @ V[:, big].T @ L1.T
    expect = L2 @ P
    assert np.linalg.norm(W[rest] - expect) <= 1e-8 * np.linalg.norm(expect)
    # the dropped directions: W(rest,:) L1 = L2 restricted to the kept right
    # singular subspace
    assert np.linalg.norm(W[rest] @ L1 - L2 @ (V[:, big] @ V[:, big].T)) <= \
        1e-8 * np.linalg.norm(L2)
