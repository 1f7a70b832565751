"""GPU parity of the single steps of Algorithm 2 against the CPU oracle:
initial norms, block sampling (bit-exact), and the robust blockwise filter."""

import numpy as np
import pytest

from oracle.cpqr import filter_block
from oracle.sampler import sample_block as oracle_sample
from workloads import adversarial_gmm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_16002_amd as rb
    rb.lib()
    return rb


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("m,n,dtype", [(1, 1, np.float64), (257, 33, np.float64),
                                       (3000, 1000, np.float32), (5000, 130, np.float32)])
def test_row_norms(rb, m, n, dtype):
    rng = np.random.default_rng(m + n)
    X = (rng.standard_normal((m, n)) * rng.uniform(0.1, 100, size=(m, 1))).astype(dtype)
    print(f"row_norms m={m} n={n} {dtype.__name__}", flush=True)
    d, s, mx = rb.row_norms(_gpu(X))
    ref = (X.astype(np.float64) ** 2).sum(1)
    dg = d.cpu().numpy()
    assert np.max(np.abs(dg - ref) / np.maximum(ref, 1e-300)) <= 4 * n * 2.0 ** -53
    assert abs(s - ref.sum()) <= 1e-13 * ref.sum()
    assert mx == pytest.approx(ref.max(), rel=1e-14)


def test_row_norms_nonfinite(rb):
    X = np.ones((100, 20), dtype=np.float32)
    X[37, 5] = np.nan
    with pytest.raises(rb.RBRPError) as e:
        rb.row_norms(_gpu(X))
    assert e.value.status == 4


def _d_cases():
    rng = np.random.default_rng(7)
    cases = []
    d = rng.exponential(size=5000)
    cases.append(("exp", d, None, 64))
    d = rng.exponential(size=20000) * 10.0 ** rng.integers(-30, 3, size=20000)
    ex = rng.uniform(size=20000) < 0.3
    cases.append(("wide+excluded", d, ex, 128))
    d = np.zeros(4097)
    d[[5, 4096, 2048, 77]] = [1.0, 2.0, 3.0, 4.0]
    cases.append(("few-positive", d, None, 16))
    d = np.zeros(300)
    d[0] = 2.0 ** 40
    d[1:40] = 1.0
    cases.append(("removal", d, None, 16))
    d = np.full(10000, 3.0)
    cases.append(("ties", d, None, 100))
    d = rng.exponential(size=2049)
    d[::3] = 0.0
    d[5] = -1e-12
    cases.append(("ragged", d, None, 1))
    return cases


@pytest.mark.parametrize("name,d,ex,b", _d_cases(), ids=[c[0] for c in _d_cases()])
def test_sampler_bit_exact(rb, name, d, ex, b):
    for t in (1, 2, 7):
        print(f"sampler case={name} t={t} b={b}", flush=True)
        got = rb.sample_block(_gpu(d), None if ex is None else _gpu(ex.astype(np.uint8)), b,
                              seed=12345, t=t, ident=3).cpu().tolist()
        want = oracle_sample(d, ex, b, seed=12345, t=t, ident=3)
        assert got == want


def _generic_block(n, nb, seed):
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((n, nb)) * rng.uniform(0.2, 5.0, size=nb)
    return V


@pytest.mark.parametrize("n,nb,seed", [(1000, 64, 1), (200, 16, 2), (40, 100, 3),
                                       (2048, 128, 4), (513, 37, 5), (7, 1, 6),
                                       (3000, 256, 7), (1500, 200, 8), (300, 160, 9),
                                       (4096, 256, 10), (129, 129, 11)])
def test_block_filter_matches_oracle(rb, n, nb, seed):
    V = _generic_block(n, nb, seed)
    # a low-rank block with noise so that the filter truncates
    if seed % 2 == 0:
        rng = np.random.default_rng(seed + 100)
        r = max(1, nb // 4)
        V = rng.standard_normal((n, r)) @ rng.standard_normal((r, nb)) + 1e-3 * V
    tau_b = 1.0 / nb
    print(f"block_cpqr n={n} nb={nb}", flush=True)
    piv, R, Qt, bp = rb.block_cpqr(_gpu(V.T), tau_b)
    opiv, oR, oQ, tails, obp = filter_block(V, tau_b)
    assert bp == obp
    assert piv.cpu().numpy()[:bp].tolist() == opiv[:bp].tolist()
    Rg = R.cpu().numpy()[:bp, :bp]
    assert np.allclose(np.abs(np.diag(Rg)), np.abs(np.diag(oR)[:bp]), rtol=1e-9, atol=0)
    Q = Qt.cpu().numpy().T                          # n x b'
    assert np.linalg.norm(Q.T @ Q - np.eye(bp)) <= 1e-13 * max(bp, 1)
    # same subspace as the oracle's kept columns
    P = oQ[:, :bp]
    assert np.linalg.norm(Q - P @ (P.T @ Q)) <= 1e-10 * np.sqrt(bp)
    # truncation identity: the kept columns reproduce V(:, piv(1:b'))
    Vs = V[:, opiv[:bp]]
    assert np.linalg.norm(Vs - Q @ (Q.T @ Vs)) <= 1e-11 * np.linalg.norm(Vs)


def test_block_filter_rank_deficient_and_orthogonal(rb):
    rng = np.random.default_rng(9)
    n, nb = 300, 32
    V = rng.standard_normal((n, 5)) @ rng.standard_normal((5, nb))
    _, _, _, bp = rb.block_cpqr(_gpu(V.T), 1.0 / nb)
    assert 1 <= bp <= 5
    Qo, _ = np.linalg.qr(rng.standard_normal((n, nb)))
    _, _, _, bp = rb.block_cpqr(_gpu(np.ascontiguousarray((2.0 * Qo).T)), 1.0 / nb)
    assert bp == nb


def test_block_filter_on_gmm_rows(rb):
    X = adversarial_gmm(3000, 256, sub_dim=64, n_comp=8, seed=3).astype(np.float64)
    V = X[:64].T.copy()
    piv, R, Qt, bp = rb.block_cpqr(_gpu(V.T), 1.0 / 64)
    opiv, _, _, _, obp = filter_block(V, 1.0 / 64)
    assert bp == obp and piv.cpu().numpy()[:bp].tolist() == opiv[:bp].tolist()


@pytest.mark.parametrize("n,nb", [(400, 48), (900, 200)])
def test_block_filter_ill_conditioned_exact_reorth(rb, n, nb):
    # condition number 1e6 with every column kept (tau_b = 0): the first basis
    # Q' = V(:, piv) R11^{-1} is orthogonal only to about u cond^2 ~ 1e-4,
    # which sends the second pass down the exact Cholesky-QR path
    rng = np.random.default_rng(nb)
    U, _ = np.linalg.qr(rng.standard_normal((n, nb)))
    Wm, _ = np.linalg.qr(rng.standard_normal((nb, nb)))
    V = U @ np.diag(np.logspace(0, -6, nb)) @ Wm
    print(f"block_cpqr ill-conditioned n={n} nb={nb}", flush=True)
    piv, R, Qt, bp = rb.block_cpqr(_gpu(V.T), 0.0)
    assert bp == nb
    Q = Qt.cpu().numpy()[:bp].T
    assert np.linalg.norm(Q.T @ Q - np.eye(bp)) <= 1e-13 * bp
    # the kept columns span exactly the columns of V
    assert np.linalg.norm(V - Q @ (Q.T @ V)) <= 1e-9 * np.linalg.norm(V)
    p = piv.cpu().numpy()
    assert sorted(p.tolist()) == list(range(nb))
    # |diag R| is the greedy sequence of residual norms: non-increasing
    dg = np.abs(np.diag(R.cpu().numpy()[:bp, :bp]))
    assert np.all(dg[1:] <= dg[:-1] * (1 + 1e-6))
