"""rbrp_id on the deflation shapes of the benchmark workloads, against the
oracle's first block and FP64 error checks.

* n = 2048, b = 128 (the power-spectrum precision-form workload's shape):
  FP32 products and the BF16 form.  n = 2048 runs the eight-wave deflation
  panels of 16 column tiles on 32-row panels with eight 16-wide b' tiles,
  in every product mode the BF16 form's controller picks (FP32 for the first
  block at eps = 1e-4, split BF16, then one BF16 product on the FP32 residual
  and finally on a BF16-stored residual).
* n = 1000, b = 64 (the adversarial GMM workload's shape) in the BF16 form:
  four-wave panels of 16 column tiles with four b' tiles.

Each run: the first block's draws, pivots and b' equal the oracle's (its
probabilities come straight from X); W(S,:) = I; the FP64 error of the
returned (S, W) meets eps; FP32: within 1.05x of the optimum on S; BF16:
the tracked residual plus the library's rounding bound E covers the optimum
on S and the true error, and the true error exceeds the optimum by at most
the stated W floor.
"""

import numpy as np
import pytest

from oracle.sampler import sample_block as oracle_sample
from oracle.cpqr import filter_block
from workloads import svd_matrix, power_spectrum, adversarial_gmm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

W_FLOOR = 5e-5    # BF16 form: true error minus the optimum on S (W from BF16-rounded L)


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_16002_amd as rb
    rb.lib()
    return rb


@pytest.fixture(scope="module")
def power2048():
    return svd_matrix(20000, 2048, power_spectrum(2048, 1.5), seed=1203).astype(np.float32)


@pytest.fixture(scope="module")
def gmm1000():
    return adversarial_gmm(20000, 1000, sub_dim=200, n_comp=50, seed=1202)


def _run(rb, Xg, eps, b, seed, **kw):
    print(f"rbrp_id m={Xg.shape[0]} n={Xg.shape[1]} eps={eps} b={b} seed={seed} {kw}",
          flush=True)
    res = rb.rbrp_id(Xg, eps, b, seed, **kw)
    torch.cuda.synchronize()
    return res


def _first_block(X, b, seed):
    X64 = X.astype(np.float64)
    d = np.einsum("ij,ij->i", X64, X64)
    idx = oracle_sample(d, None, b, seed=seed, t=1, ident=0)
    piv, _, _, _, bp = filter_block(X64[idx].T, 1.0 / b)
    return [idx[j] for j in piv[:bp]], bp


def _errors(Xg64, W, S):
    """||X - W X_S||_F / ||X||_F and the optimum on the same rows
    ||X (I - P_S)||_F / ||X||_F, FP64 on the GPU."""
    Si = torch.as_tensor(S, device=Xg64.device)
    nx = torch.linalg.norm(Xg64)
    e = torch.linalg.norm(Xg64 - W @ Xg64[Si]) / nx
    Q, _ = torch.linalg.qr(Xg64[Si].T)
    eopt = torch.linalg.norm(Xg64 - (Xg64 @ Q) @ Q.T) / nx
    return float(e), float(eopt)


def _check(rb, X, eps, b, seed, precision):
    Xg = torch.from_numpy(X).to("cuda")
    res = _run(rb, Xg, eps, b, seed, precision=precision)
    assert res.status == 0
    S = res.S.cpu().tolist()
    S1, bp1 = _first_block(X, b, seed)
    assert res.bprime[0] == bp1
    assert S[:bp1] == S1
    eye = torch.eye(res.k, dtype=torch.float64, device="cuda")
    assert torch.equal(res.W[torch.as_tensor(S, device="cuda")], eye)
    e_true, e_opt = _errors(Xg.double(), res.W, S)
    print(f"  k={res.k} blocks={res.blocks} split={res.blocks_split} "
          f"native={res.blocks_native} bf16_stored={res.blocks_bf16_stored} "
          f"e_true={e_true:.4e} e_opt={e_opt:.4e} "
          f"tracked={res.resid_tracked:.4e} E={res.err_bound:.2e}", flush=True)
    assert e_true <= eps
    assert res.resid_tracked + res.err_bound <= eps
    if precision == "native":
        assert e_true <= 1.05 * e_opt + 1e-6
        assert abs(res.resid_tracked - e_opt) <= 5e-6 + 0.02 * e_opt
    else:
        assert e_opt <= res.resid_tracked + res.err_bound
        assert abs(e_true - res.resid_tracked) <= res.err_bound
        assert e_true <= e_opt + W_FLOOR
    return res


@pytest.mark.parametrize("precision", ["native", "bf16"])
def test_n2048_b128(rb, power2048, precision):
    res = _check(rb, power2048, 1e-4, 128, 3, precision)
    assert max(res.bprime) > 64           # the eight-tile body runs
    if precision == "bf16":
        # eps = 1e-4 at the controller's budget: FP32 for the first block,
        # split BF16 while the residual is large, one product after
        assert res.blocks_native >= 1 and res.blocks_split >= 1
        assert res.blocks_native + res.blocks_split < res.blocks
        # the last blocks on a BF16-stored residual (half the bytes)
        assert res.blocks_bf16_stored >= 1


def test_n1000_b64_bf16(rb, gmm1000):
    res = _check(rb, gmm1000, 1e-3, 64, 2, "bf16")
    assert res.blocks_split >= 1 and res.blocks_native == 0
    assert res.blocks_split < res.blocks


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_bf16_error_bound_over_seeds(rb, seed):
    """The BF16 form at eps = 1e-4 on a matrix whose eps-rank (about 310) is
    well below n: the stopping rule rho + E <= eps stops early, and the true
    error stays within E of the tracked residual."""
    X = svd_matrix(20000, 512, power_spectrum(512, 2.0), seed=500 + seed).astype(np.float32)
    Xg = torch.from_numpy(X).to("cuda")
    eps = 1e-4
    res = _run(rb, Xg, eps, 64, seed, precision="bf16")
    assert res.status == 0 and res.k < 512
    S = res.S.cpu().tolist()
    e_true, e_opt = _errors(Xg.double(), res.W, S)
    print(f"  k={res.k} e_true={e_true:.4e} e_opt={e_opt:.4e} tracked={res.resid_tracked:.4e} "
          f"E={res.err_bound:.2e}", flush=True)
    assert 0.0 < res.err_bound <= 0.25 * eps
    assert abs(e_true - res.resid_tracked) <= res.err_bound
    assert e_opt <= res.resid_tracked + res.err_bound
    assert e_true <= eps
