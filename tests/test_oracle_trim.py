"""Pins for the oracle's rank trimming after Algorithm 2 (the shortest
prefix of the selection that meets the tolerance; Prop. 5.1, Alg. 3)."""

import numpy as np
import pytest

from oracle import rbrp, trim_rank, w_lstsq, w_from_l, relative_id_error
from workloads import svd_matrix, geometric_spectrum, adversarial_gmm


def _case(seed):
    s = geometric_spectrum(120, 0.9)
    return svd_matrix(400, 120, s, 30 + seed)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_trim_error_is_the_id_error_of_the_prefix(seed):
    # the projection error of the first k' basis vectors equals the optimal
    # ID error on S(1:k') (least squares, an independent route), it meets
    # eps, and one skeleton fewer does not
    X = _case(seed)
    eps = 1e-2
    res = rbrp(X, eps, 16, seed=seed)
    kt, e = trim_rank(X, res, eps)
    nx2 = float(np.sum(X * X))
    err = relative_id_error(X, w_lstsq(X, res.S[:kt]), res.S[:kt])
    assert abs(err ** 2 - e / nx2) <= 1e-10 * max(e / nx2, 1e-300)
    assert err <= eps
    prev = relative_id_error(X, w_lstsq(X, res.S[:kt - 1]), res.S[:kt - 1])
    assert prev > eps


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_trim_cuts_only_inside_the_last_block(seed):
    # the stopping rule failed at the start of the last block and the error
    # is non-increasing in the prefix length
    X = _case(seed)
    res = rbrp(X, 1e-2, 16, seed=seed)
    kt, _ = trim_rank(X, res, 1e-2)
    k_last = res.k - res.blocks[-1][1]
    assert k_last < kt <= res.k


def test_trim_removes_overshoot_somewhere():
    # large blocks overshoot: over a few seeds at least one trim is proper
    X = _case(0)
    cut = []
    for seed in range(6):
        res = rbrp(X, 1e-2, 32, seed=seed)
        kt, _ = trim_rank(X, res, 1e-2)
        cut.append(res.k - kt)
    assert max(cut) > 0 and min(cut) >= 0


def test_trim_w_is_alg3_on_leading_columns_of_l():
    # Alg. 3 on the leading k' columns of L (L_1's leading block) gives the
    # optimal W of the prefix (Prop. 5.1)
    X = adversarial_gmm(3000, 100, sub_dim=30, n_comp=8, seed=5).astype(np.float64)
    res = rbrp(X, 1e-2, 32, seed=4)
    kt, _ = trim_rank(X, res, 1e-2)
    W3 = w_from_l(res.L[:, :kt], res.S[:kt])
    Wl = w_lstsq(X, res.S[:kt])
    assert np.max(np.abs(W3 - Wl)) <= 1e-8 * max(1.0, np.max(np.abs(Wl)))


def test_trim_is_a_noop_for_single_row_blocks():
    # with b = 1 the stopping rule is checked after every skeleton
    X = _case(1)
    res = rbrp(X, 1e-2, 1, seed=3)
    kt, _ = trim_rank(X, res, 1e-2)
    assert kt == res.k


def test_trim_of_empty_selection():
    X = np.zeros((20, 6))
    res = rbrp(X, 1e-2, 4, seed=1)
    assert trim_rank(X, res, 1e-2)[0] == 0
