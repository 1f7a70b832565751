"""The C ABI loads, exports every function include/rbrp.h declares, and
rejects invalid arguments before any device work (CPU only, no GPU calls)."""

import ctypes
import os
import re

import pytest

import paper_2309_16002_amd as rb
from paper_2309_16002_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbrp.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(rbrp_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("library not built: run python -m paper_2309_16002_amd.build")
    return rb.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared_functions()
    assert "rbrp_id" in names and "rbrp_sample_block" in names
    for name in names:
        assert hasattr(L, name), name
        assert name in B.SIGNATURES, f"binding lacks {name}"


def test_status_strings(L):
    for s in range(7):
        assert isinstance(rb.status_string(s), str) and rb.status_string(s)
    assert rb.status_string(99) == "unknown status"


def test_workspace_size_is_host_only_and_validates(L):
    assert rb.workspace_size(1000, 100, 16, "f32") > 0
    assert rb.workspace_size(2000, 500, 16, "f64") > rb.workspace_size(2000, 500, 16, "f32")
    assert rb.workspace_size(0, 100, 16) == 0
    assert rb.workspace_size(100, 0, 16) == 0
    assert rb.workspace_size(100, 100, 0) == 0
    assert rb.workspace_size(100, 100, 256) > 0
    assert rb.workspace_size(100, 100, 257) == 0
    assert rb.workspace_size(100, 100, 16, k_max=101) == 0


def test_workspace_grows_with_w_refinement_steps(L):
    """The W solve's scratch in the workspace: one refinement step (the
    default) adds the A operands of the register-resident substitution to
    the plain solve's; further steps add a 64-column FP64 scratch per row
    (rows rounded up to 128)."""
    m, n, b = 50000, 600, 32
    w0, w1, w2, w3 = (rb.workspace_size(m, n, b, "f32", w_refine=r) for r in range(4))
    assert 0 < w0 < w1 < w2
    assert w2 - w1 >= 8 * 64 * m
    assert w3 == w2                                   # the scratch is reused per step
    assert rb.workspace_size(m, n, b, "f32") == w1    # one step is the default


def _call_id(L, X=1, dt=0, m=100, n=50, ldx=50, eps=0.1, b=8, S=1, k=True, W=None, ldw=0,
             ws=1, wsb=1 << 40, opt=None):
    kk = ctypes.c_int64(-7)
    st = L.rbrp_id(ctypes.c_void_p(X) if X else None, dt, m, n, ldx, eps, b, 1,
                   ctypes.byref(opt) if opt else None,
                   ctypes.c_void_p(S) if S else None, ctypes.byref(kk) if k else None,
                   ctypes.c_void_p(W) if W else None, ldw, None,
                   ctypes.c_void_p(ws) if ws else None, wsb, None)
    return st, kk.value


@pytest.mark.parametrize("kw", [
    dict(X=0), dict(S=0), dict(k=False), dict(ws=0), dict(m=0), dict(n=-1), dict(ldx=49),
    dict(eps=0.0), dict(eps=1.0), dict(eps=float("nan")), dict(b=0), dict(b=1000),
    dict(dt=7), dict(W=1, ldw=10),
])
def test_rbrp_id_rejects_invalid_arguments_without_device_work(L, kw):
    st, k = _call_id(L, **kw)
    assert st == B.RBRP_E_INVALID
    assert k == -7            # nothing written


def test_rbrp_id_workspace_too_small(L):
    st, k = _call_id(L, wsb=16)
    assert st == B.RBRP_E_WORKSPACE and k == -7


def test_bf16_needs_fp32_input(L):
    o = B.make_options(precision="bf16")
    st, _ = _call_id(L, dt=1, opt=o)
    assert st == B.RBRP_E_UNSUPPORTED


def test_hooks_validate_before_device_work(L):
    n = ctypes.c_int32(0)
    assert L.rbrp_sample_block(None, None, 10, 4, 1, 1, 0, None, ctypes.byref(n), None, 0,
                               None) == B.RBRP_E_INVALID
    assert L.rbrp_sample_block(ctypes.c_void_p(1), None, 10, 0, 1, 1, 0, ctypes.c_void_p(1),
                               ctypes.byref(n), ctypes.c_void_p(1), 1 << 30,
                               None) == B.RBRP_E_INVALID
    bp = ctypes.c_int32(0)
    assert L.rbrp_block_cpqr(ctypes.c_void_p(1), 10, 257, 10, 0.1, ctypes.c_void_p(1),
                             ctypes.c_void_p(1), ctypes.c_void_p(1), 10, ctypes.byref(bp),
                             ctypes.c_void_p(1), 1 << 30, None) == B.RBRP_E_INVALID
    assert L.rbrp_block_cpqr(ctypes.c_void_p(1), 10, 4, 10, 1.5, ctypes.c_void_p(1),
                             ctypes.c_void_p(1), ctypes.c_void_p(1), 10, ctypes.byref(bp),
                             ctypes.c_void_p(1), 1 << 30, None) == B.RBRP_E_INVALID
    s, mx = ctypes.c_double(0), ctypes.c_double(0)
    assert L.rbrp_row_norms(None, 0, 10, 10, 10, None, ctypes.byref(s), ctypes.byref(mx),
                            None, 0, None) == B.RBRP_E_INVALID
    assert L.rbrp_sample_workspace_size(0) == 0
    assert L.rbrp_block_cpqr_workspace_size(10, 0) == 0
    assert L.rbrp_row_norms_workspace_size(0) == 0


def test_no_cpu_fallback_in_binding():
    # the binding only marshals arguments: it never imports the oracle
    src = open(os.path.join(ROOT, "paper_2309_16002_amd", "_binding.py")).read()
    assert "oracle" not in src and "numpy" not in src


def _shape(m=1024, n=256, b=32, k=256, nwg=0, depth=0):
    sh = B.rbrp_batch_shape()
    sh.m_max, sh.n_max, sh.b_max, sh.k_cap_max, sh.num_wg = m, n, b, k, nwg
    sh.row_depth = depth
    return sh


def test_batch_workspace_size_validates(L):
    assert L.rbrp_batch_workspace_size(0, ctypes.byref(_shape())) > 0
    big = L.rbrp_batch_workspace_size(1, ctypes.byref(_shape()))
    assert big > L.rbrp_batch_workspace_size(0, ctypes.byref(_shape()))
    assert L.rbrp_batch_workspace_size(0, ctypes.byref(_shape(n=257))) == 0
    assert L.rbrp_batch_workspace_size(0, ctypes.byref(_shape(b=33))) == 0
    assert L.rbrp_batch_workspace_size(0, ctypes.byref(_shape(k=257))) == 0
    assert L.rbrp_batch_workspace_size(0, ctypes.byref(_shape(m=16385))) == 0
    assert L.rbrp_batch_workspace_size(2, ctypes.byref(_shape())) == 0
    assert L.rbrp_batch_workspace_size(0, None) == 0
    # row-load depth per size class: 4-bit fields of 0 (default), 1, 2 or 4
    for ok in (0x000, 0x111, 0x224, 0x421, 0x040):
        assert L.rbrp_batch_workspace_size(0, ctypes.byref(_shape(depth=ok))) > 0
    for bad in (0x003, 0x500, 0x080, 0x1000, -1):
        assert L.rbrp_batch_workspace_size(0, ctypes.byref(_shape(depth=bad))) == 0
    # scratch grows with the number of persistent workgroups
    assert (L.rbrp_batch_workspace_size(0, ctypes.byref(_shape(nwg=768)))
            > L.rbrp_batch_workspace_size(0, ctypes.byref(_shape(nwg=256))))


def _call_batched(L, descs=1, count=4, dt=0, eps=1e-3, opt=None, shape=True, k=1, st=1,
                  ws=1, wsb=1 << 40):
    sh = _shape()
    return L.rbrp_id_batched(ctypes.c_void_p(descs) if descs else None, None, count, dt, eps,
                             1, ctypes.byref(opt) if opt else None,
                             ctypes.byref(sh) if shape else None,
                             ctypes.c_void_p(k) if k else None,
                             ctypes.c_void_p(st) if st else None, None,
                             ctypes.c_void_p(ws) if ws else None, wsb, None)


def test_batched_rejects_before_device_work(L):
    # dangling non-null pointers: only host validation may run
    assert _call_batched(L, descs=0) == B.RBRP_E_INVALID
    assert _call_batched(L, k=0) == B.RBRP_E_INVALID
    assert _call_batched(L, st=0) == B.RBRP_E_INVALID
    assert _call_batched(L, ws=0) == B.RBRP_E_INVALID
    assert _call_batched(L, count=-1) == B.RBRP_E_INVALID
    assert _call_batched(L, dt=5) == B.RBRP_E_INVALID
    assert _call_batched(L, eps=-1.0) == B.RBRP_E_INVALID
    assert _call_batched(L, eps=1.0) == B.RBRP_E_INVALID
    assert _call_batched(L, shape=False) == B.RBRP_E_INVALID
    assert _call_batched(L, wsb=1) == B.RBRP_E_WORKSPACE
    assert _call_batched(L, opt=B.make_options(greedy=True)) == B.RBRP_E_UNSUPPORTED
    assert _call_batched(L, opt=B.make_options(precision="bf16")) == B.RBRP_E_UNSUPPORTED
    assert _call_batched(L, count=0) == B.RBRP_OK   # nothing to do, nothing launched


def test_batch_desc_layout():
    assert ctypes.sizeof(B.rbrp_batch_desc) == 64
    assert ctypes.sizeof(B.rbrp_batch_shape) == 32


def test_default_options_and_binding_mapping(L):
    # defaults: tau_b < 0 (-> 1/b), one W refinement step, no trimming
    o = B.rbrp_options()
    L.rbrp_default_options(ctypes.byref(o))
    assert o.tau_b < 0 and o.w_refine < 0 and o.trim == 0 and o.k_max == 0
    assert o.fixed_rank == 0 and o.greedy == 0
    # the binding: tau_b=None keeps the default, 0.0 asks for plain BRP
    assert B.make_options().tau_b < 0
    assert B.make_options(tau_b=0.0).tau_b == 0.0
    assert B.make_options(trim=True).trim == 1
    # the binding's struct has the C struct's size: rbrp_default_options
    # clears sizeof(rbrp_options) bytes of a buffer filled with 0xAB
    buf = (ctypes.c_uint8 * 256)(*([0xAB] * 256))
    L.rbrp_default_options(ctypes.cast(buf, ctypes.POINTER(B.rbrp_options)))
    c_size = max(i for i in range(256) if buf[i] != 0xAB) + 1
    assert c_size == ctypes.sizeof(B.rbrp_options) == 72
    assert B.rbrp_options.replay_d.offset == 48 and B.rbrp_options.replay_blocks.offset == 56
    assert B.rbrp_options.w_method.offset == 60 and B.rbrp_options.w_clip.offset == 64
    assert o.w_method == 0 and o.w_clip == 0.0


def test_w_method_validation(L):
    # an unknown method or a clip of 1 or more is rejected by the size query
    # and by rbrp_id before any device work
    assert rb.workspace_size(1000, 100, 16, "f32", w_method="svd") > 0
    for bad in (dict(w_method=2), dict(w_clip=1.0), dict(w_clip=float("nan"))):
        o = B.make_options()
        for key, val in bad.items():
            setattr(o, key, val)
        assert L.rbrp_workspace_size(0, 1000, 100, 16, ctypes.byref(o)) == 0
        st, k = _call_id(L, opt=o)
        assert st == B.RBRP_E_INVALID and k == -7


def test_replay_hook_validation(L):
    """replay_blocks > 0 needs the norms' pointer; a negative count is invalid
    (both rejected before any device work, k untouched)."""
    o = B.make_options()
    o.replay_blocks = 3
    st, k = _call_id(L, opt=o)
    assert st == B.RBRP_E_INVALID and k == -7
    o.replay_blocks = -1
    o.replay_d = 1
    st, k = _call_id(L, opt=o)
    assert st == B.RBRP_E_INVALID and k == -7


def test_tau_b_above_one_is_rejected_by_workspace_size(L):
    o = B.make_options(tau_b=1.5)
    assert L.rbrp_workspace_size(0, 100, 20, 8, ctypes.byref(o)) == 0
    o = B.make_options(tau_b=0.0)
    assert L.rbrp_workspace_size(0, 100, 20, 8, ctypes.byref(o)) > 0


def test_rows_beyond_the_sampler_limit_are_rejected_before_device_work(L):
    # the integer CDF has at most 4096 tiles of 2048 rows
    limit = 4096 * 2048
    assert rb.workspace_size(limit, 8, 8, "f32") > 0
    assert rb.workspace_size(limit + 1, 8, 8, "f32") == 0
    st, k = _call_id(L, m=limit + 1, n=8, ldx=8)
    assert st == B.RBRP_E_UNSUPPORTED and k == -7


def test_stats_layout():
    # blocks, blocks_split, resid_tracked, err_bound, norm_x_fro, five phase
    # times, deflate_flops, deflate_launches, blocks_native, deflate_bytes,
    # blocks_bf16_stored, w_rank, bprime[256]
    assert ctypes.sizeof(B.rbrp_stats) == 8 + 8 * 9 + 8 + 8 + 8 + 4 * 256
    assert B.rbrp_stats.err_bound.offset == 16
    assert B.rbrp_stats.deflate_bytes.offset == 88
    assert B.rbrp_stats.bprime.offset == 104


def test_sketchy_validation(L):
    """rbrp_sketchy_id: sizes and pointers checked before any device work."""
    assert L.rbrp_sketchy_workspace_size(0, 1000, 200, 50, 150) > 0
    for args in [(0, 1000, 200, 0, 150), (0, 1000, 200, 151, 150), (0, 40, 200, 50, 150),
                 (7, 1000, 200, 50, 150), (0, 1000, 200, 50, 70000), (0, 0, 200, 1, 3)]:
        assert L.rbrp_sketchy_workspace_size(*args) == 0, args
    ws = 1 << 40
    def call(X=1, k=50, l=150, Om=1, ldo=150, S=1, W=0, ldw=50, ldx=200):
        return L.rbrp_sketchy_id(ctypes.c_void_p(X) if X else None, 0, 1000, 200, ldx, k, l,
                                 ctypes.c_void_p(Om) if Om else None, ldo,
                                 ctypes.c_void_p(S) if S else None,
                                 ctypes.c_void_p(W) if W else None, ldw,
                                 ctypes.c_void_p(1), ws, None)
    for kw in (dict(X=0), dict(Om=0), dict(S=0), dict(ldo=149), dict(ldx=199),
               dict(W=1, ldw=49), dict(k=151)):
        assert call(**kw) == B.RBRP_E_INVALID, kw
    assert L.rbrp_sketchy_id(ctypes.c_void_p(1), 0, 1000, 200, 200, 50, 150, ctypes.c_void_p(1),
                             150, ctypes.c_void_p(1), None, 50, ctypes.c_void_p(1), 16,
                             None) == B.RBRP_E_WORKSPACE
