"""GPU parity of the rank trimming option of rbrp_id (the shortest prefix of
the selection whose error meets eps, then Algorithm 3 for that prefix)
against the oracle's plain definition (``oracle.trim_rank``).

FP64: the trimmed rank, the skeleton prefix and W equal the oracle's (W
within relative Frobenius error 1e-10), unless the prefix errors lie within
1e-9 of the threshold, where the two roundings may decide differently (then
only validity is checked).  FP32: the trimmed S is a prefix of the untrimmed
run's S that ends inside its last block, meets eps and is minimal, both
measured in FP64 on the GPU's own rows.
"""

import numpy as np
import pytest

from oracle import (rbrp as oracle_rbrp, trim_rank, projection_error_sq, w_lstsq,
                    relative_id_error)
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
    res = rb.rbrp_id(torch.from_numpy(np.ascontiguousarray(X)).to("cuda"), eps, b, seed, **kw)
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("m,n,b,eps,seed", [
    (400, 120, 16, 1e-2, 0), (400, 120, 16, 1e-2, 1), (400, 120, 32, 1e-2, 2),
    (1000, 300, 32, 1e-3, 2), (700, 130, 64, 1e-4, 4),
    (3000, 1000, 256, 1e-3, 5),   # b' > 128: the last block spans two deflation launches
])
def test_fp64_trim_matches_oracle(rb, m, n, b, eps, seed):
    if b > 128:
        X = svd_matrix(m, n, power_spectrum(min(m, n), 1.5), seed=1000 + m)
    else:
        X = svd_matrix(m, n, geometric_spectrum(min(m, n), 0.9), seed=1000 + m + seed)
    ref = oracle_rbrp(X, eps, b, seed)
    kt, e = trim_rank(X, ref, eps)
    full = _run(rb, X, eps, b, seed)
    res = _run(rb, X, eps, b, seed, trim=True)
    S = res.S.cpu().tolist()
    assert full.S.cpu().tolist() == ref.S
    assert S == ref.S[:res.k]
    D0 = float(np.sum(X * X))
    thr = eps * eps * D0
    near = any(abs(projection_error_sq(X, ref.Qt, j) - thr) <= 1e-9 * thr
               for j in (kt - 1, kt) if j >= 0)
    if not near:
        assert res.k == kt
        assert abs(res.resid_tracked ** 2 - e / D0) <= 1e-9 * (e / D0) + 1e-28
    W = res.W.cpu().numpy()[:, :res.k]
    Wref = w_lstsq(X, S)
    assert np.linalg.norm(W - Wref) <= 1e-10 * np.linalg.norm(Wref)
    assert np.array_equal(W[S], np.eye(res.k))
    assert relative_id_error(X, W, S) <= eps * (1 + 1e-9)
    k_last = ref.k - ref.blocks[-1][1]
    assert k_last < res.k <= full.k


@pytest.mark.parametrize("m,n,b,seed", [(6000, 250, 32, 1), (20000, 1000, 64, 2)])
def test_fp32_trim_is_a_minimal_prefix(rb, m, n, b, seed):
    eps = 1e-3
    X = adversarial_gmm(m, n, sub_dim=min(200, n // 2), n_comp=20, seed=seed)
    full = _run(rb, X, eps, b, seed)
    res = _run(rb, X, eps, b, seed, trim=True)
    Sf = full.S.cpu().tolist()
    S = res.S.cpu().tolist()
    assert S == Sf[:res.k]
    assert full.k - full.bprime[-1] < res.k <= full.k
    Xg = torch.from_numpy(X.astype(np.float64)).to("cuda")
    nx = torch.linalg.norm(Xg)

    def err(rows):
        Q, _ = torch.linalg.qr(Xg[torch.as_tensor(rows, device="cuda")].T)
        return float(torch.linalg.norm(Xg - (Xg @ Q) @ Q.T) / nx)

    # meets eps and one row fewer does not (FP32 tracking: 1e-3 relative slack)
    assert err(S) <= eps * (1 + 1e-3)
    assert err(S[:-1]) > eps * (1 - 1e-3)
    W = res.W[:, :res.k]
    e = float(torch.linalg.norm(Xg - W @ Xg[torch.as_tensor(S, device="cuda")]) / nx)
    assert e <= 1.05 * err(S) + 1e-6
    assert abs(res.resid_tracked - err(S)) <= 5e-6 + 0.02 * err(S)


def test_trim_ignored_with_fixed_rank(rb):
    X = svd_matrix(400, 120, geometric_spectrum(120, 0.9), seed=77)
    a = _run(rb, X, 0.5, 16, 3, k_max=37, fixed_rank=True)
    t = _run(rb, X, 0.5, 16, 3, k_max=37, fixed_rank=True, trim=True)
    assert a.k == t.k == 37
    assert a.S.cpu().tolist() == t.S.cpu().tolist()


def test_trim_ignored_in_bf16_form(rb):
    X = adversarial_gmm(6000, 250, sub_dim=125, n_comp=20, seed=1)
    a = _run(rb, X, 1e-3, 32, 1, precision="bf16")
    t = _run(rb, X, 1e-3, 32, 1, precision="bf16", trim=True)
    assert a.k == t.k
    assert a.S.cpu().tolist() == t.S.cpu().tolist()
