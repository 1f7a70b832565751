"""The interpolation matrix through the truncated-SVD pseudo-inverse of L_1
(Remark 5.2, rbrp_options.w_method = 1) against the oracle's w_svd_pinv.

* FP64, no truncation: the same skeletons as the oracle, W within 1e-10 of
  the oracle's pseudo-inverse W and of least squares; every singular value kept.
* FP64 with truncation: a spectrum of 20 unit values and a flat tail at 1e-10
  run to eps = 1e-12 selects the tail rows too; the relative clip 1e-7 drops
  exactly the tail's singular values on both sides (a factor 100 from the
  clip), and W matches the oracle's within 1e-10.
* FP32: the pseudo-inverse W and the substitution W of the same run agree to
  rounding, and the decomposition meets eps; k = 203 and 512 (several
  values per thread in the Jacobi rotations, odd and even k).
"""

import numpy as np
import pytest

from oracle import rbrp as oracle_rbrp, w_lstsq, w_svd_pinv, relative_id_error
from workloads import svd_matrix, geometric_spectrum, power_spectrum, adversarial_gmm

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
    Xg = torch.from_numpy(np.ascontiguousarray(X)).to("cuda")
    res = rb.rbrp_id(Xg, eps, b, seed, **kw)
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("seed", [1, 2])
def test_fp64_no_truncation_matches_oracle(rb, seed):
    X = svd_matrix(2000, 500, geometric_spectrum(500, 0.9), seed=1001)
    res = _run(rb, X, 1e-2, 16, seed, w_method="svd")
    ref = oracle_rbrp(X, 1e-2, 16, seed)
    assert res.S.cpu().tolist() == ref.S
    Wref, kept = w_svd_pinv(ref.L, ref.S, clip=1e-12)
    assert kept == ref.k and res.w_rank == ref.k
    W = res.W.cpu().numpy()
    assert np.array_equal(W[ref.S], np.eye(ref.k))
    assert np.linalg.norm(W - Wref) <= 1e-10 * np.linalg.norm(Wref)
    Wl = w_lstsq(X, ref.S)
    assert np.linalg.norm(W - Wl) <= 1e-10 * np.linalg.norm(Wl)


def test_fp64_truncation_matches_oracle(rb):
    s = np.concatenate([np.ones(20), np.full(180, 1e-10)])
    X = svd_matrix(1000, 200, s, seed=77)
    eps, b, seed, clip = 1e-12, 16, 4, 1e-7
    res = _run(rb, X, eps, b, seed, w_method="svd", w_clip=clip)
    ref = oracle_rbrp(X, eps, b, seed)
    assert ref.k > 20
    assert res.S.cpu().tolist() == ref.S
    sv = np.linalg.svd(np.tril(ref.L[ref.S]), compute_uv=False)
    # the clip sits in a wide gap of L_1's spectrum
    kept_ref = int(np.count_nonzero(sv >= clip * sv[0]))
    assert kept_ref == 20
    assert sv[kept_ref - 1] >= 100 * clip * sv[0] and sv[kept_ref] <= 1e-2 * clip * sv[0]
    Wref, kept = w_svd_pinv(ref.L, ref.S, clip=clip)
    assert kept == 20 and res.w_rank == 20
    W = res.W.cpu().numpy()
    assert np.linalg.norm(W - Wref) <= 1e-10 * np.linalg.norm(Wref)
    # dropping the tail directions costs about the tail's share of ||X||
    e = relative_id_error(X, W, ref.S)
    tail = np.linalg.norm(s[20:]) / np.linalg.norm(s)
    print(f"  k={res.k} kept={res.w_rank} ID error {e:.3e} (tail {tail:.3e})", flush=True)
    assert e <= 1.5 * tail


@pytest.mark.parametrize("case", ["gmm_20000x1000", "power_20000x512"])
def test_fp32_pinv_equals_substitution(rb, case):
    if case == "gmm_20000x1000":
        X = adversarial_gmm(20000, 1000, sub_dim=200, n_comp=50, seed=1402)
        eps, b = 1e-3, 64
    else:
        X = svd_matrix(20000, 512, power_spectrum(512, 1.5), seed=1403).astype(np.float32)
        eps, b = 1e-4, 32
    a = _run(rb, X, eps, b, 5)
    p = _run(rb, X, eps, b, 5, w_method="svd")
    assert a.status == 0 and p.status == 0
    assert torch.equal(a.S, p.S)
    assert p.w_rank == p.k
    d = torch.linalg.norm(a.W - p.W) / torch.linalg.norm(a.W)
    Xg = torch.from_numpy(X).to("cuda").double()
    e = float(torch.linalg.norm(Xg - p.W @ Xg[p.S]) / torch.linalg.norm(Xg))
    print(f"  k={p.k} |W_svd - W_sub| / |W_sub| = {float(d):.2e}, ID error {e:.3e}", flush=True)
    assert float(d) <= 1e-9
    assert e <= eps
