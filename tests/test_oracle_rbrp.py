"""Pins for the oracle's Algorithm 2 loop and interpolation matrix
(Alg. 2, Alg. 1, Alg. 3, Prop. 5.1, eq. stable_id, eq. skeletonization_error)."""

import numpy as np
import pytest
import scipy.linalg

from oracle import rbrp, srp, w_lstsq, w_from_l, relative_id_error
from workloads import (svd_matrix, geometric_spectrum, power_spectrum, exact_rank,
                       adversarial_gmm, gmm_example41, example23)


def _cfg1_small(m=400, n=120, q=0.9, seed=21):
    s = geometric_spectrum(n, q)
    return svd_matrix(m, n, s, seed), s


@pytest.mark.parametrize("form", ["A", "B"])
def test_tracked_residual_is_skeletonization_error(form):
    # Prop. 5.1: ||d||_1 = ||X - L Q^T||_F^2 = E_X(S) = min_W ||X - W X_S||_F^2
    X, _ = _cfg1_small()
    r = rbrp(X, 1e-2, 16, seed=1, form=form)
    assert r.k > 0
    e_lq = np.linalg.norm(X - r.L @ r.Qt) ** 2
    W = w_lstsq(X, r.S)
    e_skel = np.linalg.norm(X - W @ X[r.S]) ** 2
    assert abs(r.resid_sq - e_skel) <= 1e-10 * e_skel
    assert abs(e_lq - e_skel) <= 1e-10 * e_skel


def test_stopping_rule_tau_is_eps_squared():
    # stop at the first block boundary where ||d||_1 <= eps^2 ||d^(0)||_1
    X, _ = _cfg1_small()
    eps = 3e-2
    r = rbrp(X, eps, 8, seed=2)
    assert r.rho <= eps
    k_before = r.k - r.blocks[-1][1]
    W = w_lstsq(X, r.S[:k_before])
    assert relative_id_error(X, W, r.S[:k_before]) > eps


def test_basis_orthonormal_and_spans_skeletons():
    X, _ = _cfg1_small()
    r = rbrp(X, 1e-3, 16, seed=3)
    k = r.k
    assert np.linalg.norm(r.Qt @ r.Qt.T - np.eye(k)) <= 1e-14 * k
    XS = X[r.S]
    assert np.linalg.norm(XS - (XS @ r.Qt.T) @ r.Qt) <= 1e-13 * np.linalg.norm(XS)


def test_alg3_w_equals_optimal_w():
    # Alg. 3 / Prop. 5.1: W(S,:) = I and W = L L_1^{-1} = X X_S^+
    X, _ = _cfg1_small()
    r = rbrp(X, 1e-2, 16, seed=4)
    W3 = w_from_l(r.L, r.S)
    Wl = w_lstsq(X, r.S)
    assert np.array_equal(W3[r.S], np.eye(r.k))
    assert np.linalg.norm(W3 - Wl) <= 1e-10 * np.linalg.norm(Wl)
    # W X_S = L Q^T (Prop. 5.1)
    assert np.linalg.norm(W3 @ X[r.S] - r.L @ r.Qt) <= 1e-10 * np.linalg.norm(X)


def test_l1_is_lower_triangular():
    X, _ = _cfg1_small()
    r = rbrp(X, 1e-3, 16, seed=5)
    L1 = r.L[r.S, :]
    assert np.linalg.norm(np.triu(L1, 1)) <= 1e-13 * np.linalg.norm(L1)
    # diagonal entries of a kept pivot are nonzero
    assert np.min(np.abs(np.diag(L1))) > 0


@pytest.mark.parametrize("r_true,b", [(5, 16), (12, 8), (40, 16), (7, 1)])
def test_exact_recovery_on_exact_rank(r_true, b):
    # a matrix of exact rank r is recovered with k = r and no error
    X = exact_rank(300, 90, r_true, seed=30 + r_true)
    res = rbrp(X, 1e-6, b, seed=6)
    assert res.k == r_true
    W = w_lstsq(X, res.S)
    assert relative_id_error(X, W, res.S) <= 1e-12


def test_exact_recovery_example23():
    # Example 2.3: the k scaled canonical directions recover X exactly
    r, beta, alpha = 3, 2, 1e4
    k = (1 + beta) * r
    X = example23(12 * k, k, r, alpha)
    res = rbrp(X, 1e-8, 4, seed=7)
    assert res.k == k
    assert sorted(int(np.flatnonzero(X[i])[0]) for i in res.S) == list(range(k))


def test_b1_is_sequential_random_pivoting():
    # b = 1: the filter keeps the single sampled row (tau_b = 1), so RBRP is
    # Algorithm 1 (independent rank-one implementation, same random stream)
    X, _ = _cfg1_small(m=300, n=80)
    res = rbrp(X, 5e-2, 1, seed=8)
    S, L, d, D0 = srp(X, 5e-2, seed=8)
    assert res.S == S
    assert abs(res.resid_sq - d.sum()) <= 1e-10 * D0
    # Alg. 1 alone: its downdated residual is the skeletonization error
    W = w_lstsq(X, S)
    e = np.linalg.norm(X - W @ X[S]) ** 2
    assert abs(d.sum() - e) <= 1e-9 * e
    assert np.linalg.norm(w_from_l(L, S) - W) <= 1e-9 * np.linalg.norm(W)


def test_greedy_b1_is_lapack_cpqr_of_xt():
    # Remark 4.3: top-1 greedy selection is CPQR on X^T (LAPACK dgeqp3)
    rng = np.random.default_rng(9)
    X = rng.standard_normal((60, 25)) * rng.uniform(0.5, 2.0, size=(60, 1))
    res = rbrp(X, 1e-12, 1, seed=0, greedy=True, k_max=25, fixed_rank=True)
    _, _, piv = scipy.linalg.qr(X.T, mode="economic", pivoting=True)
    assert res.S == [int(p) for p in piv[:25]]


def test_forms_a_and_b_select_same_skeletons():
    X = adversarial_gmm(4000, 120, sub_dim=40, n_comp=10, seed=11).astype(np.float64)
    ra = rbrp(X, 1e-3, 32, seed=9, form="A")
    rb = rbrp(X, 1e-3, 32, seed=9, form="B")
    assert ra.S == rb.S
    assert abs(ra.resid_sq - rb.resid_sq) <= 1e-9 * ra.D0


def test_eckart_young_lower_bound():
    # ||d||_1 >= sum_{i > k} sigma_i^2 for the prescribed spectrum
    m, n = 500, 150
    s = power_spectrum(n, 1.5)
    X = svd_matrix(m, n, s, seed=12)
    res = rbrp(X, 1e-2, 16, seed=10)
    assert res.resid_sq >= (s[res.k:] ** 2).sum() * (1 - 1e-12)


def test_config1_rank_bounds():
    # the svd-geometric workload (2000 x 500, s_i = 0.9^i, eps = 1e-2): the
    # optimal rank is 44 (eta_44 <= 1e-4 < eta_43), so k >= 44
    s = geometric_spectrum(500, 0.9)
    tail = np.cumsum((s ** 2)[::-1])[::-1] / (s ** 2).sum()
    r_star = int(np.argmax(np.append(tail[1:], 0.0) <= 1e-4)) + 1
    assert r_star == 44
    X = svd_matrix(2000, 500, s, seed=1001)
    res = rbrp(X, 1e-2, 16, seed=1)
    assert 44 <= res.k <= 44 + 40
    assert res.rho <= 1e-2


def test_zero_matrix_and_kmax():
    X = np.zeros((30, 10))
    res = rbrp(X, 1e-2, 4, seed=1)
    assert res.k == 0 and res.S == []
    X, _ = _cfg1_small()
    res = rbrp(X, 1e-6, 16, seed=1, k_max=20)
    assert res.k == 20
    res = rbrp(X, 0.5, 16, seed=1, k_max=37, fixed_rank=True)
    assert res.k == 37


def test_rbrp_filter_beats_brp_on_example41():
    # Example 4.1 / Conjecture 4.4: robust filtering (tau_b = 1/b) needs fewer
    # skeletons than plain BRP (tau_b = 0) on the GMM pitfall matrix
    X = gmm_example41(n_clusters=40, cluster_size=25, n=200, seed=13)
    ks_r, ks_p = [], []
    for seed in range(4):
        ks_r.append(rbrp(X, 0.1, 20, seed=seed).k)
        ks_p.append(rbrp(X, 0.1, 20, seed=seed, tau_b=0.0).k)
    assert np.mean(ks_r) < np.mean(ks_p)
