"""Pins for the oracle's sketchy pivoting (SkLUPP) and oversampled sketchy ID
(OSID, Algorithm 4).

* The pivots equal LAPACK's partial-pivoting LU (scipy.linalg.lu_factor) on
  the sketch's first k columns, including a case with repeated rows (ties go
  to the first row, as LAPACK's idamax).
* OSID's W equals Y Y_S^+ computed by least squares, and W(S,:) = I.
* With a square orthogonal embedding (l = n) the sketch loses nothing:
  Omega Omega^+ = I, so OSID's W is the optimal X X_S^+ (eq. stable_id).
* On a matrix of exact rank k the sketchy ID is exact.
"""

import numpy as np
import pytest
import scipy.linalg

from oracle import w_lstsq, relative_id_error
from oracle.sketchy import sketch, lupp_pivots, osid, sketchy_id
from workloads import svd_matrix, gaussian_exp, exact_rank, haar


def _lapack_pivots(Y, k):
    _, ipiv = scipy.linalg.lu_factor(Y[:, :k])
    perm = np.arange(Y.shape[0])
    for i, p in enumerate(ipiv):
        perm[i], perm[p] = perm[p], perm[i]
    return [int(x) for x in perm[:k]]


@pytest.mark.parametrize("shape", [(300, 40, 40), (500, 60, 25), (64, 64, 64)])
def test_pivots_equal_lapack_getrf(shape):
    m, l, k = shape
    Y = np.random.default_rng(m + l + k).standard_normal((m, l))
    assert lupp_pivots(Y, k) == _lapack_pivots(Y, k)


def test_pivot_ties_go_to_the_first_row():
    rng = np.random.default_rng(3)
    base = rng.standard_normal((50, 12))
    Y = np.vstack([base, base[::-1]])     # every row twice
    assert lupp_pivots(Y, 12) == _lapack_pivots(Y, 12)
    assert all(p < 50 for p in lupp_pivots(Y, 1))


def test_osid_is_y_times_pinv_of_y_s():
    X = gaussian_exp(400, 300, seed=5)
    Omega = np.random.default_rng(6).standard_normal((300, 90))
    S, W, Y = sketchy_id(X, Omega, 30)
    assert np.array_equal(W[S], np.eye(30))
    Wt, *_ = np.linalg.lstsq(Y[S].T, Y.T, rcond=None)
    rest = np.setdiff1d(np.arange(400), S)
    assert np.linalg.norm(W[rest] - Wt.T[rest]) <= 1e-10 * np.linalg.norm(Wt.T[rest])


def test_square_orthogonal_embedding_gives_the_optimal_w():
    X = svd_matrix(300, 80, np.linspace(1.0, 0.01, 80), seed=9)
    Omega = haar(np.random.default_rng(10), 80, 80)
    S, W, _ = sketchy_id(X, Omega, 25)
    Wopt = w_lstsq(X, S)
    assert np.linalg.norm(W - Wopt) <= 1e-10 * np.linalg.norm(Wopt)


def test_exact_rank_is_recovered():
    X = exact_rank(500, 120, 20, seed=12)
    Omega = np.random.default_rng(13).standard_normal((120, 60))
    S, W, _ = sketchy_id(X, Omega, 20)
    assert relative_id_error(X, W, S) <= 1e-12
