"""Sketchy pivoting (LU with partial pivoting on Y = X Omega) and the
oversampled sketchy interpolation matrix (Algorithm 4) through the C ABI,
against the oracle on the same embedding Omega.

* Gaussian-exp (section 6's 1000 x 1000 matrix, FP64) and an adversarial GMM
  matrix (20000 x 1000, FP32 promoted exactly): the skeletons equal the
  oracle's pivot rows element by element; W matches the oracle's OSID W to
  1e-10 relative; W(S,:) = I.
* k = 1, 32 (one whole panel), 100 and 150 (several panels and a ragged last
  one); l = 3k as in the paper, and l = k (no oversampling).
* Skeletons only (W = NULL) gives the same S.
"""

import numpy as np
import pytest

from oracle.sketchy import sketchy_id as oracle_sketchy
from oracle import relative_id_error
from workloads import gaussian_exp, adversarial_gmm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_16002_amd as rb
    rb.lib()
    return rb


@pytest.fixture(scope="module")
def gexp():
    return gaussian_exp(1000, 1000, seed=1006)


@pytest.fixture(scope="module")
def gmm():
    return adversarial_gmm(20000, 1000, sub_dim=200, n_comp=50, seed=1502)


def _check(rb, X, k, l, seed, want_w=True):
    n = X.shape[1]
    Omega = np.random.default_rng(seed).standard_normal((n, l))
    print(f"sketchy_id m={X.shape[0]} n={n} {X.dtype} k={k} l={l} seed={seed} w={want_w}",
          flush=True)
    Xg = torch.from_numpy(np.ascontiguousarray(X)).to("cuda")
    Og = torch.from_numpy(Omega).to("cuda")
    S, W = rb.sketchy_id(Xg, Og, k, want_w=want_w)
    torch.cuda.synchronize()
    S = S.cpu().tolist()
    S_ref, W_ref, _ = oracle_sketchy(np.asarray(X, dtype=np.float64), Omega, k)
    first = next((i for i, (a, b) in enumerate(zip(S, S_ref)) if a != b), None)
    assert S == S_ref, f"first difference at {first}"
    if want_w:
        Wn = W.cpu().numpy()
        assert np.array_equal(Wn[S], np.eye(k))
        d = np.linalg.norm(Wn - W_ref) / np.linalg.norm(W_ref)
        e = relative_id_error(np.asarray(X, dtype=np.float64), Wn, S)
        print(f"  |W - W_oracle| / |W_oracle| = {d:.2e}, ID error {e:.3e}", flush=True)
        assert d <= 1e-10
    return S


@pytest.mark.parametrize("k,over", [(1, 3), (32, 3), (100, 3), (150, 3), (100, 1)])
def test_gaussian_exp_fp64(rb, gexp, k, over):
    _check(rb, gexp, k, over * k, seed=10 + k)


@pytest.mark.parametrize("k", [64, 128])
def test_gmm_fp32(rb, gmm, k):
    _check(rb, gmm, k, 3 * k, seed=20 + k)


def test_skeletons_only(rb, gexp):
    a = _check(rb, gexp, 70, 210, seed=5, want_w=False)
    b = _check(rb, gexp, 70, 210, seed=5, want_w=True)
    assert a == b
