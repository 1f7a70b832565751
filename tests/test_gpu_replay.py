"""Skeleton parity beyond the first block: the GPU run fed the oracle's
residual norms.

With the replay hook of rbrp_options, block t of the GPU run draws from the
squared residual row norms the FP64 oracle drew from in its block t (the
Philox stream, the integer weights and the exclusion of rows already in S
are the library's own).  The sampled rows, their projection on the basis and
the robust filter are FP64 from the original rows of X in both, so with the
same norms every block must select the same rows and the same b', whatever
precision the GPU's deflation used: S is compared end to end, element by
element, in FP64, FP32 and the BF16 form.

A second test runs both sides free (the GPU's own FP32/BF16 norms) over ten
seeds and reports the ratio of the ranks k_GPU / k_oracle; the median must lie
within 5 % of 1.
"""

import statistics

import numpy as np
import pytest

from oracle import rbrp as oracle_rbrp, relative_id_error
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


@pytest.fixture(scope="module")
def gmm20k():
    return adversarial_gmm(20000, 1000, sub_dim=200, n_comp=50, seed=1302)


@pytest.fixture(scope="module")
def power2048():
    return svd_matrix(20000, 2048, power_spectrum(2048, 1.5), seed=1303).astype(np.float32)


def _replay(rb, X, eps, b, seed, precision):
    """The oracle run with its per-block norms, then the GPU run replaying them."""
    X64 = np.asarray(X, dtype=np.float64)
    trace = []
    ref = oracle_rbrp(X64, eps, b, seed, trace=trace)
    D = torch.from_numpy(np.ascontiguousarray(np.stack(trace))).to("cuda")
    Xg = torch.from_numpy(np.ascontiguousarray(X)).to("cuda")
    print(f"replay m={X.shape[0]} n={X.shape[1]} {X.dtype} eps={eps} b={b} seed={seed} "
          f"{precision}: oracle k={ref.k} blocks={len(ref.blocks)}", flush=True)
    res = rb.rbrp_id(Xg, eps, b, seed, precision=precision, replay_d=D)
    torch.cuda.synchronize()
    return ref, res


def _assert_same(ref, res):
    S = res.S.cpu().tolist()
    assert res.status == 0
    assert res.blocks == len(ref.blocks)
    assert res.bprime == [bp for _, bp in ref.blocks]
    first_diff = next((i for i, (a, c) in enumerate(zip(S, ref.S)) if a != c), None)
    assert S == ref.S, f"first difference at position {first_diff} of {len(ref.S)}"


@pytest.mark.parametrize("seed", [1, 2])
def test_replay_fp64(rb, seed):
    X = svd_matrix(2000, 500, geometric_spectrum(500, 0.9), seed=1001)
    ref, res = _replay(rb, X, 1e-2, 16, seed, "native")
    _assert_same(ref, res)
    W = res.W.cpu().numpy()
    assert relative_id_error(X, W, ref.S) <= 1e-2


@pytest.mark.parametrize("precision", ["native", "bf16"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_replay_fp32_gmm(rb, gmm20k, precision, seed):
    ref, res = _replay(rb, gmm20k, 1e-3, 64, seed, precision)
    assert len(ref.blocks) >= 3
    _assert_same(ref, res)


@pytest.mark.parametrize("precision", ["native", "bf16"])
def test_replay_fp32_power_n2048_b128(rb, power2048, precision):
    ref, res = _replay(rb, power2048, 1e-4, 128, 3, precision)
    assert len(ref.blocks) >= 10
    _assert_same(ref, res)


def _k_ratios(rb, X, eps, b, seeds, precision, cache):
    Xg = torch.from_numpy(np.ascontiguousarray(X)).to("cuda")
    X64 = np.asarray(X, dtype=np.float64)
    ratios = []
    for seed in seeds:
        if seed not in cache:
            cache[seed] = oracle_rbrp(X64, eps, b, seed, form="A").k
        res = rb.rbrp_id(Xg, eps, b, seed, precision=precision, want_w=False)
        torch.cuda.synchronize()
        assert res.status == 0
        ratios.append(res.k / cache[seed])
    return ratios


_ORACLE_K = {}


@pytest.fixture(scope="module")
def gmm100k():
    return adversarial_gmm(100000, 1000, seed=1002)


@pytest.mark.parametrize("case", ["gmm_100000x1000", "power_20000x2048"])
@pytest.mark.parametrize("precision", ["native", "bf16"])
def test_rank_ratio_over_ten_seeds(rb, request, case, precision):
    if case == "gmm_100000x1000":
        X, eps, b = request.getfixturevalue("gmm100k"), 1e-3, 64
    else:
        X, eps, b = request.getfixturevalue("power2048"), 1e-4, 128
    cache = _ORACLE_K.setdefault(case, {})
    print(f"k ratio {case} {precision}", flush=True)
    r = _k_ratios(rb, X, eps, b, range(10), precision, cache)
    med = statistics.median(r)
    print(f"  k_GPU/k_oracle per seed {[round(x, 4) for x in r]} median {med:.4f}", flush=True)
    assert 0.95 <= med <= 1.05
