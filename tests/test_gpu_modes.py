"""GPU parity of the selection-mode options of rbrp_id against the oracle:
plain BRP (tau_b = 0: no robust filter, the paper's blockwise random
pivoting), blockwise greedy pivoting (RBGP, Remark 4.3) with b > 1, and an
explicit tau_b equal to the default 1/b.  FP64 inputs of full numerical rank
per block: skeletons and b' identical, W within 1e-10 of least squares;
plain BRP on numerically rank-deficient blocks: the pivots up to the rank
identical, both IDs exact to rounding."""

import numpy as np
import pytest

from oracle import rbrp as oracle_rbrp, w_lstsq, relative_id_error
from workloads import svd_matrix, geometric_spectrum, adversarial_gmm, exact_rank

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_16002_amd as rb
    rb.lib()
    return rb


def _run(rb, X, eps, b, seed, **kw):
    print(f"rbrp_id m={X.shape[0]} n={X.shape[1]} {X.dtype} eps={eps} b={b} seed={seed} {kw}",
          flush=True)
    res = rb.rbrp_id(torch.from_numpy(np.ascontiguousarray(X)).to("cuda"), eps, b, seed, **kw)
    torch.cuda.synchronize()
    return res


def _check(res, ref, X, eps):
    S = res.S.cpu().tolist()
    assert S == ref.S
    assert res.bprime == [bp for _, bp in ref.blocks]
    W = res.W.cpu().numpy()
    Wref = w_lstsq(X, S)
    assert np.linalg.norm(W - Wref) <= 1e-10 * np.linalg.norm(Wref)
    assert relative_id_error(X, W, S) <= eps * (1 + 1e-9)


@pytest.mark.parametrize("m,n,b,eps,seed", [(400, 120, 16, 1e-2, 1), (1000, 300, 32, 1e-3, 2)])
def test_plain_brp_matches_oracle(rb, m, n, b, eps, seed):
    X = svd_matrix(m, n, geometric_spectrum(min(m, n), 0.9), seed=2000 + m)
    ref = oracle_rbrp(X, eps, b, seed, tau_b=0.0)
    res = _run(rb, X, eps, b, seed, tau_b=0.0)
    _check(res, ref, X, eps)
    # no filter: every block but a final short one keeps all b rows
    assert all(bp == b for bp in res.bprime[:-1])


@pytest.mark.parametrize("m,n,r,b,seed", [(2000, 300, 10, 16, 1), (2000, 300, 20, 32, 2),
                                          (3000, 200, 40, 64, 3), (2000, 300, 10, 16, 4)])
def test_plain_brp_rank_deficient_blocks(rb, m, n, r, b, seed):
    """Plain BRP on a matrix of exact rank r < b, so the first block is
    numerically rank-deficient.  The oracle's Householder CPQR keeps all b
    columns (the last b - r on rounding noise); the GPU's pivoted Cholesky of
    the Gram matrix keeps pivoting while the remaining diagonal is positive,
    so it keeps the r columns and at most the few noise columns before the
    first non-positive diagonal.  Both give an exact ID: the first r pivots
    agree, W(S,:) = I and the error is at the rounding level."""
    X = exact_rank(m, n, r, seed=700 + seed)
    eps = 1e-8
    ref = oracle_rbrp(X, eps, b, seed, tau_b=0.0)
    res = _run(rb, X, eps, b, seed, tau_b=0.0)
    assert res.status == 0
    assert ref.k == b and len(res.bprime) == 1
    S = res.S.cpu().tolist()
    assert S[:r] == ref.S[:r]
    assert r <= res.k <= b
    W = res.W.cpu().numpy()
    assert np.array_equal(W[S], np.eye(res.k))
    e = relative_id_error(X, W, S)
    print(f"  b'={res.k} (oracle {ref.k}), error {e:.2e}, max|W| {np.abs(W).max():.2e}",
          flush=True)
    assert e <= 1e-13
    assert np.abs(W).max() <= 1e3


@pytest.mark.parametrize("m,n,b,eps", [
    (400, 120, 16, 1e-2), (1500, 200, 8, 1e-3),
    (5000, 150, 32, 1e-2),    # more than one 2048-row chunk: two selection passes
    (20000, 100, 64, 1e-2),   # ten chunks, then a pass over their kept keys
    (5000, 150, 1, 1e-2),     # b = 1: the argmax path over three chunks
])
def test_greedy_blocks_match_oracle(rb, m, n, b, eps):
    X = svd_matrix(m, n, geometric_spectrum(min(m, n), 0.9), seed=3000 + m)
    ref = oracle_rbrp(X, eps, b, 0, greedy=True)
    res = _run(rb, X, eps, b, 0, greedy=True)
    _check(res, ref, X, eps)


def test_explicit_tau_b_equals_default(rb):
    X = adversarial_gmm(3000, 120, sub_dim=40, n_comp=10, seed=3).astype(np.float64)
    a = _run(rb, X, 1e-3, 32, 4)
    t = _run(rb, X, 1e-3, 32, 4, tau_b=1.0 / 32)
    assert a.S.cpu().tolist() == t.S.cpu().tolist()
    assert a.bprime == t.bprime


def test_tau_b_above_one_is_rejected(rb):
    X = np.ones((50, 10))
    with pytest.raises(rb.RBRPError):
        _run(rb, X, 1e-2, 4, 0, tau_b=1.5)


@pytest.mark.parametrize("eps,seed", [(1e-2, 1), (1e-3, 2)])
def test_b1_is_sequential_random_pivoting(rb, eps, seed):
    # Alg. 1 (SRP): one row per step, drawn in proportion to the residual's
    # squared row norms; the oracle's independent SRP code
    from oracle import srp
    X = svd_matrix(300, 80, geometric_spectrum(80, 0.85), seed=4000 + seed)
    S_ref, _, _, _ = srp(X, eps, seed)
    res = _run(rb, X, eps, 1, seed)
    S = res.S.cpu().tolist()
    assert S == list(S_ref)
    W = res.W.cpu().numpy()
    Wref = w_lstsq(X, S)
    assert np.linalg.norm(W - Wref) <= 1e-10 * np.linalg.norm(Wref)
