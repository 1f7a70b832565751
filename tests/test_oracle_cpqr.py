"""Pins for the oracle's local CPQR and robust blockwise filtering
(Alg. 2 local CPQR and truncation; Remark 4.2; rationale of Conjecture 4.4)."""

import itertools
import math

import numpy as np
import pytest
import scipy.linalg

from oracle.cpqr import cpqr, filter_block, tails_from_r, truncation_rank


@pytest.mark.parametrize("n,b,seed", [(60, 16, 0), (200, 64, 1), (10, 24, 2), (300, 8, 3)])
def test_pivots_match_lapack_geqp3(n, b, seed):
    # generic V (no near ties): same pivot order and |diag R| as LAPACK's
    # column-pivoted QR (dgeqp3 via scipy).
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((n, b)) * rng.uniform(0.1, 10.0, size=b)
    piv, R, Q = cpqr(V)
    _, R2, piv2 = scipy.linalg.qr(V, mode="economic", pivoting=True)
    r = min(n, b)
    assert list(piv[:r]) == list(piv2[:r])
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(R2)), rtol=1e-12, atol=0)
    assert np.linalg.norm(V[:, piv] - Q @ R) <= 1e-13 * np.linalg.norm(V)
    assert np.linalg.norm(Q.T @ Q - np.eye(r)) <= 1e-14 * r


def test_each_pivot_is_brute_force_greedy():
    # eq. qr_update: pivot p is the column farthest from span(chosen), found
    # here by an independent least-squares distance for every candidate.
    rng = np.random.default_rng(4)
    n, b = 30, 10
    V = rng.standard_normal((n, 4)) @ rng.standard_normal((4, b)) + 0.3 * rng.standard_normal((n, b))
    piv, _, _ = cpqr(V)
    chosen = []
    for p in range(b):
        best, best_j = -1.0, None
        for j in range(b):
            if j in chosen:
                continue
            if chosen:
                A = V[:, chosen]
                coef, *_ = np.linalg.lstsq(A, V[:, j], rcond=None)
                dist = np.linalg.norm(V[:, j] - A @ coef)
            else:
                dist = np.linalg.norm(V[:, j])
            if dist > best:
                best, best_j = dist, j
        assert piv[p] == best_j
        chosen.append(best_j)


def test_ties_go_to_lowest_sampled_position():
    rng = np.random.default_rng(5)
    v = rng.standard_normal(20)
    w = rng.standard_normal(20)
    V = np.column_stack([0.5 * w, v, w * 0.1, v])   # columns 1 and 3 identical
    piv, _, _ = cpqr(V)
    assert piv[0] == 1


def test_truncation_identity_remark42():
    # ||V(:,pi) - Q_V(:,1:b') R_V(1:b',:)||_F^2 = ||R_V(b'+1:, b'+1:)||_F^2 < tau_b ||V||_F^2
    rng = np.random.default_rng(6)
    n, b = 80, 16
    V = rng.standard_normal((n, 5)) @ rng.standard_normal((5, b)) * 3 + rng.standard_normal((n, b)) * 0.05
    piv, R, Q, tails, bp = filter_block(V, 1.0 / b)
    lhs = np.linalg.norm(V[:, piv] - Q[:, :bp] @ R[:bp, :]) ** 2
    rhs = np.sum(R[bp:, bp:] ** 2)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(V ** 2)
    assert rhs < np.sum(V ** 2) / b
    # b' is the largest index meeting the threshold
    assert tails[bp - 1] >= np.sum(V ** 2) / b
    assert bp == b or np.all(tails[bp:] < np.sum(V ** 2) / b)


def test_rank_deficient_block_keeps_at_most_rank():
    # rationale of Conjecture 4.4: rank(V) = b'' < b gives b' <= b''
    rng = np.random.default_rng(7)
    n, b = 50, 12
    for rank in (1, 3, 7):
        V = rng.standard_normal((n, rank)) @ rng.standard_normal((rank, b))
        *_, bp = filter_block(V, 1.0 / b)
        assert 1 <= bp <= rank


def test_orthogonal_equal_norm_columns_keep_all():
    # rationale of Conjecture 4.4: orthogonal columns of equal norm give b' = b
    rng = np.random.default_rng(8)
    for n, b in ((40, 16), (64, 64), (100, 7)):
        Qo, _ = np.linalg.qr(rng.standard_normal((n, b)))
        *_, bp = filter_block(Qo * 2.5, 1.0 / b)
        assert bp == b


def test_b_larger_than_n():
    rng = np.random.default_rng(9)
    V = rng.standard_normal((5, 12))
    piv, R, Q, tails, bp = filter_block(V, 1.0 / 12)
    assert R.shape == (5, 12) and Q.shape == (5, 5)
    assert np.all(tails[5:] == 0) and bp <= 5


def _vol(V, cols):
    if not cols:
        return 1.0
    return math.sqrt(max(np.linalg.det(V[:, list(cols)].T @ V[:, list(cols)]), 0.0))


def test_best_subset_on_constructed_tiny_blocks():
    # For orthogonal columns of distinct norms greedy pivoting is optimal: the
    # kept subset is the maximum-volume subset of its size (brute force).
    rng = np.random.default_rng(10)
    for b in (3, 4, 5, 6):
        Qo, _ = np.linalg.qr(rng.standard_normal((12, b)))
        norms = rng.permutation(np.linspace(1.0, 3.0, b))
        V = Qo * norms
        piv, _, _, _, bp = filter_block(V, 1.0 / b)
        got = set(int(p) for p in piv[:bp])
        best = max(itertools.combinations(range(b), bp), key=lambda c: _vol(V, c))
        assert got == set(best)
    # a duplicated direction is never kept twice
    for b in (4, 5, 6):
        base = rng.standard_normal((10, b - 1))
        V = np.column_stack([base, base[:, 0] * 0.999])
        piv, _, _, _, bp = filter_block(V, 1.0 / b)
        kept = set(int(p) for p in piv[:bp])
        assert not {0, b - 1} <= kept


def test_greedy_volume_bound_on_random_tiny_blocks():
    # the greedy subset's volume is within a factor k! of the best subset
    # (the classical guarantee for greedy volume maximisation).
    rng = np.random.default_rng(11)
    for trial in range(20):
        b = int(rng.integers(3, 7))
        V = rng.standard_normal((8, b)) * rng.uniform(0.2, 2.0, size=b)
        piv, _, _ = cpqr(V)
        for k in range(1, b + 1):
            g = _vol(V, [int(p) for p in piv[:k]])
            best = max(_vol(V, c) for c in itertools.combinations(range(b), k))
            assert g >= best / math.factorial(k) * (1 - 1e-12)


def test_tails_from_r_is_trailing_frobenius():
    R = np.triu(np.arange(1.0, 17.0).reshape(4, 4))
    tails = tails_from_r(R, 4)
    for i in range(4):
        assert tails[i] == sum(R[l, j] ** 2 for l in range(i, 4) for j in range(l, 4))
    assert truncation_rank(tails, 0.25, 4) == max(i + 1 for i in range(4) if tails[i] >= 0.25 * tails[0] * (1 - 16 * 2.0 ** -53))
