"""End-to-end GPU parity of rbrp_id (Algorithm 2 + Algorithm 3) against the
CPU FP64 oracle.

Tolerances: FP64 results within relative Frobenius error 1e-10 of the
oracle.  FP32 ("plain" single-precision deflation) cannot reproduce the FP64
sampling probabilities bit for bit once the residual has been deflated in
FP32 (d carries relative errors of order u32 ||x_i|| / ||r_i||), so the
FP32 checks are: the first block is identical (its d comes straight from X),
the tracked residual equals the true interpolation error of the returned
(S, W) to the FP32 floor, W matches X X_S^+ on the GPU's own S, W(S,:) = I,
and the error meets eps.
"""

import numpy as np
import pytest

from oracle import rbrp as oracle_rbrp, w_lstsq, relative_id_error
from workloads import (svd_matrix, geometric_spectrum, power_spectrum, exact_rank,
                       adversarial_gmm, config_matrix)

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


def _run(rb, X, eps, b, seed, **kw):
    print(f"rbrp_id m={X.shape[0]} n={X.shape[1]} {X.dtype} eps={eps} b={b} seed={seed} {kw}",
          flush=True)
    res = rb.rbrp_id(_gpu(X), eps, b, seed, **kw)
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("m,n,b,eps,seed", [
    (400, 120, 16, 1e-2, 1), (1000, 300, 32, 1e-3, 2), (333, 77, 8, 1e-2, 3),
    (2000, 500, 16, 1e-2, 1),   # the svd-geometric FP64 workload at full size
    (700, 130, 64, 1e-4, 4),
    (3000, 1000, 256, 1e-3, 5),  # b > 128: global-memory filter, two deflation launches
    (1500, 400, 200, 1e-4, 6),   # ... and a run that ends at full rank (k = n)
    (2500, 1300, 64, 1e-3, 7),   # 1024 < n <= 2048: eight-wave deflation panels
    (1200, 300, 32, 1e-4, 8),    # n padded to 384: the filter products in three K slices
])
def test_fp64_matches_oracle(rb, m, n, b, eps, seed):
    if b > 128:
        X = svd_matrix(m, n, power_spectrum(min(m, n), 1.5 if n >= 1000 else 1.0),
                       seed=1000 + m)
    else:
        X = svd_matrix(m, n, geometric_spectrum(min(m, n), 0.9), seed=1000 + m)
    res = _run(rb, X, eps, b, seed)
    ref = oracle_rbrp(X, eps, b, seed)
    assert res.S.cpu().tolist() == ref.S
    assert res.bprime == [bp for _, bp in ref.blocks]
    W = res.W.cpu().numpy()
    Wref = w_lstsq(X, ref.S)
    assert np.linalg.norm(W - Wref) <= 1e-10 * np.linalg.norm(Wref)
    assert np.array_equal(W[ref.S], np.eye(res.k))
    # relative 1e-10, with an absolute floor at rounding level for runs that
    # end at full rank (rho ~ 1e-16)
    assert abs(res.resid_tracked - ref.rho) <= 1e-10 * ref.rho + 1e-14
    e_true = relative_id_error(X, W, ref.S)
    assert abs(e_true - res.resid_tracked) <= 1e-9 * e_true + 1e-14
    assert e_true <= 1.05 * relative_id_error(X, Wref, ref.S)
    if b > 128:
        assert max(res.bprime) > 128


@pytest.mark.parametrize("m,n,b,eps,seed", [
    (1, 7, 16, 1e-12, 1),     # one row
    (7, 1, 4, 1e-12, 2),      # one column
    (10, 40, 16, 1e-12, 3),   # fewer rows than b: the whole matrix in one block
    (40, 10, 64, 1e-12, 4),   # b > m and b > n
    (16, 16, 16, 1e-3, 5),    # m = n = b
    (65, 17, 8, 1e-12, 6),    # ragged rows and columns, run to full rank
    (129, 33, 32, 1e-3, 7),
    (3, 300, 2, 1e-12, 8),    # the filter keeps one of two columns per block
])
def test_fp64_tiny_and_degenerate_shapes(rb, m, n, b, eps, seed):
    """Gaussian matrices of tiny and degenerate shapes against the oracle:
    the same skeletons and block sizes, W = X X_S^+ to 1e-10 (with an
    absolute floor: several runs end at full rank, where W(rest,:) is exact
    up to rounding), W(S,:) = I."""
    X = np.random.default_rng(seed).standard_normal((m, n))
    res = _run(rb, X, eps, b, seed)
    ref = oracle_rbrp(X, eps, b, seed)
    assert res.status == 0
    assert res.S.cpu().tolist() == ref.S
    assert res.bprime == [bp for _, bp in ref.blocks]
    W = res.W.cpu().numpy()
    Wref = w_lstsq(X, ref.S)
    assert np.array_equal(W[ref.S], np.eye(res.k))
    assert np.linalg.norm(W - Wref) <= 1e-10 * np.linalg.norm(Wref) + 1e-12
    assert abs(res.resid_tracked - ref.rho) <= 1e-10 * ref.rho + 1e-14


@pytest.mark.parametrize("r,b", [(5, 16), (40, 16), (12, 8), (70, 32)])
def test_fp64_exact_rank_recovery(rb, r, b):
    X = exact_rank(600, 150, r, seed=40 + r)
    res = _run(rb, X, 1e-6, b, 3)
    assert res.k == r
    W = res.W.cpu().numpy()
    assert relative_id_error(X, W, res.S.cpu().tolist()) <= 1e-12


def test_fp64_kmax_capacity_and_fixed_rank(rb):
    X = svd_matrix(500, 100, geometric_spectrum(100, 0.95), seed=8)
    res = _run(rb, X, 1e-6, 16, 1, k_max=30)
    assert res.k == 30 and res.status == 5
    ref = oracle_rbrp(X, 1e-6, 16, 1, k_max=30)
    assert res.S.cpu().tolist() == ref.S
    res = _run(rb, X, 0.5, 16, 1, k_max=37, fixed_rank=True)
    ref = oracle_rbrp(X, 0.5, 16, 1, k_max=37, fixed_rank=True)
    assert res.k == 37 and res.S.cpu().tolist() == ref.S


@pytest.mark.parametrize("refine", [0, 1, 2])
def test_fp64_w_solve_refinement_steps(rb, refine):
    """W by blocked substitution (Alg. 3) over several 64-wide column blocks
    with a ragged last block: W matches X X_S^+ on the same S with and without
    refinement steps."""
    X = svd_matrix(3000, 400, geometric_spectrum(400, 0.97), seed=77)
    res = _run(rb, X, 1e-4, 32, 2, w_refine=refine)
    S = res.S.cpu().tolist()
    assert res.k > 192 and res.k % 64 != 0
    W = res.W.cpu().numpy()
    Wref = w_lstsq(X, S)
    tol = 1e-10 if refine > 0 else 1e-9
    assert np.linalg.norm(W - Wref) <= tol * np.linalg.norm(Wref)
    assert np.array_equal(W[S], np.eye(res.k))


@pytest.mark.parametrize("k", [1, 64, 65, 128])
def test_fp64_w_solve_block_boundaries(rb, k):
    """Fixed rank k at and around the 64-column blocks of the substitution
    (one column; exactly one block; one block plus one column; two blocks):
    W matches X X_S^+ and W(S,:) = I."""
    X = svd_matrix(1500, 300, geometric_spectrum(300, 0.98), seed=79)
    res = _run(rb, X, 1e-12, 16, 4, k_max=k, fixed_rank=True)
    assert res.k == k
    S = res.S.cpu().tolist()
    W = res.W.cpu().numpy()
    Wref = w_lstsq(X, S)
    assert np.linalg.norm(W - Wref) <= 1e-10 * np.linalg.norm(Wref)
    assert np.array_equal(W[S], np.eye(k))


@pytest.mark.parametrize("k", [129, 200, 256, 257, 320, 513, 259])
def test_fp64_w_solve_super_blocks(rb, k):
    """Fixed rank k within and around the 256-column super-blocks of the
    solve (two and a ragged third and fourth column block of one
    super-block; one whole super-block; one plus one column; a ragged second;
    three; an odd k = k_max = 259, whose rows of W are loaded element by
    element by the tall GEMM): the later super-blocks' contribution goes
    through the tall GEMM into W's columns, and W still matches X X_S^+ with
    W(S,:) = I."""
    X = svd_matrix(2500, 600, geometric_spectrum(600, 0.99), seed=81)
    res = _run(rb, X, 1e-12, 32, 5, k_max=k, fixed_rank=True)
    assert res.k == k
    S = res.S.cpu().tolist()
    W = res.W.cpu().numpy()
    Wref = w_lstsq(X, S)
    assert np.linalg.norm(W - Wref) <= 1e-10 * np.linalg.norm(Wref)
    assert np.array_equal(W[S], np.eye(k))


@pytest.mark.parametrize("k", [20, 40, 104, 148, 350])
def test_fp64_w_solve_partial_last_block(rb, k):
    """Fixed rank k whose last 64-column block holds two or three 16-column
    tiles (20, 148: 20 columns; 40, 104: 40; 350: a second super-block of 94
    columns whose last block has 30): the products of that block run in
    their two- and three-tile forms, and W still matches X X_S^+ with
    W(S,:) = I."""
    X = svd_matrix(2500, 600, geometric_spectrum(600, 0.99), seed=83)
    res = _run(rb, X, 1e-12, 32, 6, k_max=k, fixed_rank=True)
    assert res.k == k
    S = res.S.cpu().tolist()
    W = res.W.cpu().numpy()
    Wref = w_lstsq(X, S)
    assert np.linalg.norm(W - Wref) <= 1e-10 * np.linalg.norm(Wref)
    assert np.array_equal(W[S], np.eye(k))


def test_fp64_w_solve_odd_leading_dimension(rb):
    """k = k_max = 131 (an odd leading dimension of W: the element-wise load
    path of the substitution) at fixed rank."""
    X = svd_matrix(2000, 300, geometric_spectrum(300, 0.98), seed=78)
    res = _run(rb, X, 1e-12, 16, 3, k_max=131, fixed_rank=True)
    assert res.k == 131 and res.W.shape[1] == 131
    S = res.S.cpu().tolist()
    W = res.W.cpu().numpy()
    Wref = w_lstsq(X, S)
    assert np.linalg.norm(W - Wref) <= 1e-10 * np.linalg.norm(Wref)
    assert np.array_equal(W[S], np.eye(131))


def test_fp32_w_refinement_step(rb):
    """FP32 input: the default solve (one fused refinement step) and the
    plain substitution give the same skeletons, and W to far below the FP32
    rounding of L; the refined W is at least as close to X X_S^+."""
    X = adversarial_gmm(20000, 500, sub_dim=200, n_comp=20, seed=5)
    a = _run(rb, X, 1e-3, 64, 4, w_refine=0)
    b = _run(rb, X, 1e-3, 64, 4)
    S = b.S.cpu().tolist()
    assert a.S.cpu().tolist() == S
    Wa, Wb = a.W.cpu().numpy(), b.W.cpu().numpy()
    assert np.linalg.norm(Wa - Wb) <= 1e-9 * np.linalg.norm(Wb)
    assert np.array_equal(Wb[S], np.eye(b.k))
    X64 = X.astype(np.float64)
    e_b = relative_id_error(X64, Wb, S)
    assert e_b <= 1.05 * relative_id_error(X64, w_lstsq(X64, S), S) + 1e-6


def test_zero_matrix(rb):
    res = _run(rb, np.zeros((100, 40)), 1e-2, 8, 1)
    assert res.k == 0


def test_nonfinite_input(rb):
    X = np.ones((64, 32), dtype=np.float32)
    X[3, 3] = np.inf
    with pytest.raises(rb.RBRPError) as e:
        _run(rb, X, 1e-2, 8, 1)
    assert e.value.status == 4


def test_deterministic(rb):
    X = adversarial_gmm(5000, 200, sub_dim=50, n_comp=10, seed=4)
    a = _run(rb, X, 1e-3, 32, 9)
    b = _run(rb, X, 1e-3, 32, 9)
    assert a.S.cpu().tolist() == b.S.cpu().tolist()
    assert torch.equal(a.W, b.W)


@pytest.mark.parametrize("m,n,b,seed", [(6000, 250, 32, 1), (20000, 1000, 64, 2),
                                        (8000, 1500, 64, 3)])
def test_fp32_adversarial_gmm(rb, m, n, b, seed):
    eps = 1e-3
    X = adversarial_gmm(m, n, sub_dim=min(200, n // 2), n_comp=20, seed=seed)
    res = _run(rb, X, eps, b, seed)
    ref = oracle_rbrp(X.astype(np.float64), eps, b, seed)
    S = res.S.cpu().tolist()
    # first block: identical draws and filter (d^(0) comes straight from X)
    bp0 = ref.blocks[0][1]
    assert res.bprime[0] == bp0
    assert S[:bp0] == ref.S[:bp0]
    X64 = X.astype(np.float64)
    W = res.W.cpu().numpy()
    assert np.array_equal(W[S], np.eye(res.k))
    e_true = relative_id_error(X64, W, S)
    Wopt = w_lstsq(X64, S)
    e_opt = relative_id_error(X64, Wopt, S)
    # stated FP32 bound: interpolation error within 1.05x of the optimum on S
    # and the eps target met
    assert e_true <= 1.05 * e_opt + 1e-6
    assert e_true <= eps * 1.01
    # tracked residual vs the true residual: FP32 floor
    assert abs(res.resid_tracked - e_opt) <= 5e-6 + 0.02 * e_opt
    # skeleton count close to the oracle's at the same eps
    assert abs(res.k - ref.k) <= max(b, 0.15 * ref.k)


def test_fp32_svd_matches_oracle_skeletons_mostly(rb):
    X = svd_matrix(3000, 400, power_spectrum(400, 1.5), seed=31).astype(np.float32)
    res = _run(rb, X, 1e-2, 32, 5)
    ref = oracle_rbrp(X.astype(np.float64), 1e-2, 32, 5)
    S = res.S.cpu().tolist()
    W = res.W.cpu().numpy()
    e = relative_id_error(X.astype(np.float64), W, S)
    assert e <= 1e-2 * 1.01
    assert S[:ref.blocks[0][1]] == ref.S[:ref.blocks[0][1]]


def test_greedy_b1_matches_oracle(rb):
    rng = np.random.default_rng(9)
    X = rng.standard_normal((300, 60)) * rng.uniform(0.5, 2.0, size=(300, 1))
    res = _run(rb, X, 1e-12, 1, 0, greedy=True, k_max=40, fixed_rank=True)
    ref = oracle_rbrp(X, 1e-12, 1, 0, greedy=True, k_max=40, fixed_rank=True)
    assert res.S.cpu().tolist() == ref.S


def _true_errors_gpu(Xg, W, S):
    """||X - W X_S||_F / ||X||_F and the optimum on the same rows,
    ||X (I - P_S)||_F / ||X||_F, in FP64 on the GPU."""
    Si = torch.as_tensor(S, device=Xg.device)
    nx = torch.linalg.norm(Xg)
    e = torch.linalg.norm(Xg - W[:, :len(S)] @ Xg[Si]) / nx
    Q, _ = torch.linalg.qr(Xg[Si].T)
    eopt = torch.linalg.norm(Xg - (Xg @ Q) @ Q.T) / nx
    return float(e), float(eopt)


@pytest.mark.parametrize("precision", ["native", "bf16"])
def test_fp32_random_features_b256(rb, precision):
    """The large random-feature workload (cos(x Omega + c), n = 4096, b = 256)
    at m = 100000 rows.  Its eps-rank at 1e-3 is close to n, so the workload
    runs to a fixed rank k = 2048 (the "or k" stopping rule).  The first
    block against the oracle's sampler and filter; the error bounds of the
    whole run in FP64."""
    from oracle.sampler import sample_block as oracle_sample
    from oracle.cpqr import filter_block
    eps, b, seed, k = 1e-3, 256, 5, 2048
    X = config_matrix("random_features_large", m=100000)
    res = _run(rb, X, eps, b, seed, precision=precision, k_max=k, fixed_rank=True)
    S = res.S.cpu().tolist()
    assert res.k == k and res.status == 0
    assert max(res.bprime) > 128
    X64 = X.astype(np.float64)
    d = np.einsum("ij,ij->i", X64, X64)
    idx = oracle_sample(d, None, b, seed=seed, t=1, ident=0)
    opiv, _, _, _, obp = filter_block(X64[idx].T, 1.0 / b)
    assert res.bprime[0] == obp
    assert S[:obp] == [idx[j] for j in opiv[:obp]]
    Xg = torch.from_numpy(X64).to("cuda")
    del X64
    W = res.W
    assert torch.equal(W[torch.as_tensor(S, device="cuda")][:, :res.k],
                       torch.eye(res.k, dtype=torch.float64, device="cuda"))
    e_true, e_opt = _true_errors_gpu(Xg, W, S)
    print(f"  k={res.k} blocks={len(res.bprime)} e_true={e_true:.4e} e_opt={e_opt:.4e} "
          f"tracked={res.resid_tracked:.4e}", flush=True)
    if precision == "native":
        assert e_true <= 1.05 * e_opt + 1e-6
        assert abs(res.resid_tracked - e_opt) <= 5e-6 + 0.02 * e_opt
    else:
        assert e_true <= e_opt + 5e-5 + res.err_bound
