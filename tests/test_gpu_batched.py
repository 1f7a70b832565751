"""Batched form (rbrp_id_batched): many independent IDs in one persistent
launch, checked ID by ID against the CPU oracle run with the same Philox
counter word (the ID's index in the batch).

FP64 batches reproduce the oracle's skeletons exactly and W to 1e-10.  FP32
batches (residual and products in FP32, norms / basis / W in FP64) reproduce
the first block exactly and meet eps, with the stated FP32 floor for the
tracked residual (the single-ID FP32 bound).  The launch is capture-safe:
a HIP graph of it replays to the same outputs.
"""

import numpy as np
import pytest

from oracle import rbrp as oracle_rbrp, w_lstsq, relative_id_error
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


def _fp64_batch(count, seed0):
    rng = np.random.default_rng(seed0)
    Xs = []
    for i in range(count):
        m = int(rng.integers(40, 500))
        n = int(rng.integers(20, 160))
        q = float(rng.uniform(0.75, 0.95))
        Xs.append(svd_matrix(m, n, geometric_spectrum(min(m, n), q), seed=seed0 + i))
    return Xs


def _launch(rb, Xs, eps, b, seed, **kw):
    print(f"rbrp_id_batched count={len(Xs)} eps={eps} b={b} seed={seed} {kw}", flush=True)
    Xg = [torch.from_numpy(np.ascontiguousarray(X)).to("cuda") for X in Xs]
    plan = rb.BatchPlan(Xg, b=b, num_wg=kw.pop("num_wg", 0))
    rb.rbrp_id_batched(plan, eps, seed, **kw)
    torch.cuda.synchronize()
    return plan


@pytest.mark.parametrize("b", [8, 12, 16])
def test_fp64_batch_matches_oracle(rb, b):
    eps, seed = 1e-3, 5
    Xs = _fp64_batch(24, 300 + b)
    plan = _launch(rb, Xs, eps, b, seed)
    for i, X in enumerate(Xs):
        S, k, W, status, resid = plan.result(i)
        ref = oracle_rbrp(X, eps, b, seed, ident=i)
        assert status == 0, (i, status)
        assert S.cpu().tolist() == ref.S, i
        Wn = W.cpu().numpy()
        Wref = w_lstsq(X, ref.S)
        assert np.linalg.norm(Wn - Wref) <= 1e-10 * np.linalg.norm(Wref), i
        assert np.array_equal(Wn[ref.S], np.eye(k))
        # IDs that reach full rank end at rounding level: absolute floor
        assert abs(resid - ref.rho) <= 1e-10 * ref.rho + 1e-14, i


def test_fp32_kernel_blocks(rb):
    eps, b, seed = 1e-6, 16, 3
    Xs = kernel_blocks(count=48, m_range=(64, 600), n_range=(32, 200), seed=44)
    plan = _launch(rb, Xs, eps, b, seed)
    for i, X in enumerate(Xs):
        S, k, W, status, resid = plan.result(i)
        assert status == 0, (i, status)
        S = S.cpu().tolist()
        X64 = X.astype(np.float64)
        ref = oracle_rbrp(X64, eps, b, seed, ident=i)
        bp0 = ref.blocks[0][1]
        assert S[:bp0] == ref.S[:bp0], i
        Wn = W.cpu().numpy()
        assert np.array_equal(Wn[S], np.eye(k))
        e_true = relative_id_error(X64, Wn, S)
        e_opt = relative_id_error(X64, w_lstsq(X64, S), S)
        assert e_true <= eps * 1.01 + 3e-7, (i, e_true)
        assert e_true <= 1.05 * e_opt + 3e-7, i
        assert abs(resid - e_opt) <= 3e-7 + 0.02 * e_opt, i
        assert abs(k - ref.k) <= max(b, 0.2 * ref.k), i


def test_batch_invalid_descriptor_is_isolated(rb):
    Xs = _fp64_batch(4, 900)
    Xg = [torch.from_numpy(X).to("cuda") for X in Xs]
    plan = rb.BatchPlan(Xg, b=8)
    # corrupt ID 2's descriptor on the device: k_cap beyond min(m, n)
    d = plan.descs_host[2]
    d.k_cap = min(d.m, d.n) + 1
    plan.descs = torch.frombuffer(bytearray(bytes(plan.descs_host)),
                                  dtype=torch.uint8).to("cuda")
    rb.rbrp_id_batched(plan, 1e-3, 1)
    torch.cuda.synchronize()
    st = plan.status_out.cpu().tolist()
    assert st[2] == 1 and plan.k_out[2].item() == 0
    assert st[0] == st[1] == st[3] == 0


def test_batch_graph_replay(rb):
    eps, b, seed = 1e-6, 16, 2
    Xs = kernel_blocks(count=32, m_range=(64, 400), n_range=(32, 128), seed=45)
    Xg = [torch.from_numpy(X).to("cuda") for X in Xs]
    plan = rb.BatchPlan(Xg, b=b)
    rb.rbrp_id_batched(plan, eps, seed)
    torch.cuda.synchronize()
    S0, W0, k0 = plan.S_all.clone(), plan.W_all.clone(), plan.k_out.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            rb.rbrp_id_batched(plan, eps, seed)
    torch.cuda.synchronize()
    for rep in range(3):
        plan.S_all.fill_(-1)
        plan.W_all.fill_(float("nan"))
        plan.k_out.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(plan.k_out, k0), rep
        for i in range(plan.count):
            k = int(k0[i])
            a, c = plan.s_off[i], plan.w_off[i]
            assert torch.equal(plan.S_all[a:a + k], S0[a:a + k]), (rep, i)
            Wi = plan.W_all[c:plan.w_off[i + 1]].view(plan.ms[i], plan.ks[i])[:, :k]
            Wr = W0[c:plan.w_off[i + 1]].view(plan.ms[i], plan.ks[i])[:, :k]
            assert torch.equal(Wi, Wr), (rep, i)


def test_batch_autotune(rb):
    eps, seed = 1e-6, 7
    Xs = kernel_blocks(count=64, m_range=(64, 700), n_range=(32, 256), seed=46)
    Xg = [torch.from_numpy(X).to("cuda") for X in Xs]
    plan = rb.BatchPlan(Xg, b=16)
    bcls = rb.batch_autotune(plan, eps, seed)
    print("autotuned b per class", bcls, "num_wg", plan.shape.num_wg, flush=True)
    assert all(x in (0, 8, 16, 32) for x in bcls) and any(bcls)
    assert plan.shape.num_wg in (256, 512, 768)
    order = plan.order.cpu().tolist()
    assert sorted(order) == list(range(plan.count))
    rb.rbrp_id_batched(plan, eps, seed)
    torch.cuda.synchronize()
    for i, X in enumerate(Xs):
        S, k, W, status, resid = plan.result(i)
        assert status == 0
        S = S.cpu().tolist()
        X64 = X.astype(np.float64)
        assert relative_id_error(X64, W.cpu().numpy(), S) <= eps * 1.01 + 3e-7, i
