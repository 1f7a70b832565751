"""rbrp_id_batched_noalloc (the batched form on the library's static scratch
array, for callers that cannot allocate) against rbrp_id_batched on a
caller-provided workspace: the same kernels, so every output is compared
for equality (k, status, S, W, tracked residual), ID by ID.

Two calls in a row, the second on a smaller batch: the array keeps the first
call's contents, so the second call shows that nothing is read before it is
written.  The FP32 batch's largest IDs (m up to 1000, n up to 256) need more
scratch per workgroup than 512 workgroups of the array hold, so it also runs
the reduced persistent grid.
"""

import numpy as np
import pytest

from workloads import svd_matrix, geometric_spectrum, kernel_blocks

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_16002_amd as rb
    rb.lib()
    return rb


def _fp64_batch(count, seed0, m_hi, n_hi):
    rng = np.random.default_rng(seed0)
    Xs = []
    for i in range(count):
        m = int(rng.integers(40, m_hi))
        n = int(rng.integers(20, n_hi))
        q = float(rng.uniform(0.75, 0.95))
        Xs.append(svd_matrix(m, n, geometric_spectrum(min(m, n), q), seed=seed0 + i))
    return Xs


def _plans(rb, Xs, b):
    Xg = [torch.from_numpy(np.ascontiguousarray(X)).to("cuda") for X in Xs]
    return Xg, rb.BatchPlan(Xg, b=b), rb.BatchPlan(Xg, b=b)


def _same(pa, pb):
    torch.cuda.synchronize()
    assert torch.equal(pa.k_out, pb.k_out)
    assert torch.equal(pa.status_out, pb.status_out)
    assert torch.equal(pa.resid_out, pb.resid_out)
    for i in range(pa.count):
        Sa, ka, Wa, sa, _ = pa.result(i)
        Sb, kb, Wb, sb, _ = pb.result(i)
        assert sa == 0 and ka == kb, i
        assert torch.equal(Sa, Sb), i
        assert torch.equal(Wa, Wb), i


def _run_pair(rb, Xs, eps, b, seed):
    print(f"batch count={len(Xs)} m_max={max(X.shape[0] for X in Xs)} "
          f"n_max={max(X.shape[1] for X in Xs)} dtype={Xs[0].dtype} eps={eps} b={b}",
          flush=True)
    Xg, pa, pb = _plans(rb, Xs, b)
    rb.rbrp_id_batched(pa, eps, seed)
    rb.rbrp_id_batched_noalloc(pb, eps, seed)
    _same(pa, pb)
    return pa


def test_noalloc_matches_workspace_fp64_twice(rb):
    # first call: 24 IDs up to 500 x 160; second: 9 smaller IDs
    _run_pair(rb, _fp64_batch(24, 900, 500, 160), 1e-3, 16, 5)
    _run_pair(rb, _fp64_batch(9, 950, 120, 60), 1e-3, 8, 6)


def test_noalloc_matches_workspace_fp32_reduced_grid(rb):
    Xs = kernel_blocks(count=40, m_range=(64, 1000), n_range=(32, 256), seed=71)
    pa = _run_pair(rb, Xs, 1e-6, 16, 3)
    assert int(pa.k_out.min()) >= 1
    # a smaller FP32 batch right after, on the same array
    _run_pair(rb, kernel_blocks(count=12, m_range=(64, 300), n_range=(32, 96), seed=72),
              1e-6, 16, 4)


def test_noalloc_rejects_shape_beyond_limits(rb):
    """Every shape within the batched form's limits fits the array (the
    largest, 16384 x 256 with k_cap 256 in FP64, needs about 66 MiB per
    workgroup); a shape beyond them is rejected before any device work (the
    outputs keep their sentinel values)."""
    Xg = [torch.ones((64, 32), dtype=torch.float32, device="cuda")]
    plan = rb.BatchPlan(Xg, b=8)
    plan.shape.m_max = 16385
    plan.k_out.fill_(-5)
    torch.cuda.synchronize()
    with pytest.raises(rb.RBRPError) as ei:
        rb.rbrp_id_batched_noalloc(plan, 1e-3, 0)
    assert ei.value.status == 1     # RBRP_E_INVALID
    torch.cuda.synchronize()
    assert int(plan.k_out[0]) == -5
