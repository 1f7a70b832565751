"""ctypes binding of the RBRP C ABI (include/rbrp.h).

Argument marshalling only: PyTorch provides device memory (outputs and the
workspace) and the current stream; every step of the decomposition runs in
the library's HIP kernels.  The library must have been built
(``paper_2309_16002_amd.build``); nothing here falls back to other code.
"""

import ctypes
import os
from dataclasses import dataclass

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "librbrp.so")

RBRP_OK = 0
RBRP_E_INVALID = 1
RBRP_E_WORKSPACE = 2
RBRP_E_HIP = 3
RBRP_E_NONFINITE = 4
RBRP_E_CAPACITY = 5
RBRP_E_UNSUPPORTED = 6

RBRP_F32 = 0
RBRP_F64 = 1
PRECISIONS = {"native": 0, "bf16": 1}


class rbrp_options(ctypes.Structure):
    _fields_ = [
        ("tau_b", ctypes.c_double),
        ("k_max", ctypes.c_int64),
        ("fixed_rank", ctypes.c_int32),
        ("greedy", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("w_refine", ctypes.c_int32),
        ("theta", ctypes.c_double),
        ("profile", ctypes.c_int32),
        ("trim", ctypes.c_int32),
        ("replay_d", ctypes.c_void_p),
        ("replay_blocks", ctypes.c_int32),
        ("w_method", ctypes.c_int32),
        ("w_clip", ctypes.c_double),
    ]


class rbrp_stats(ctypes.Structure):
    _fields_ = [
        ("blocks", ctypes.c_int32),
        ("blocks_split", ctypes.c_int32),
        ("resid_tracked", ctypes.c_double),
        ("err_bound", ctypes.c_double),
        ("norm_x_fro", ctypes.c_double),
        ("ms_init", ctypes.c_double),
        ("ms_select", ctypes.c_double),
        ("ms_filter", ctypes.c_double),
        ("ms_deflate", ctypes.c_double),
        ("ms_interp", ctypes.c_double),
        ("deflate_flops", ctypes.c_double),
        ("deflate_launches", ctypes.c_int32),
        ("blocks_native", ctypes.c_int32),
        ("deflate_bytes", ctypes.c_double),
        ("blocks_bf16_stored", ctypes.c_int32),
        ("w_rank", ctypes.c_int32),
        ("bprime", ctypes.c_int32 * 256),
    ]


class rbrp_batch_desc(ctypes.Structure):
    _fields_ = [
        ("X", ctypes.c_void_p),
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("ldx", ctypes.c_int64),
        ("S", ctypes.c_void_p),
        ("W", ctypes.c_void_p),
        ("ldw", ctypes.c_int64),
        ("k_cap", ctypes.c_int32),
        ("b", ctypes.c_int32),
    ]


class rbrp_batch_shape(ctypes.Structure):
    _fields_ = [
        ("m_max", ctypes.c_int64),
        ("n_max", ctypes.c_int64),
        ("b_max", ctypes.c_int32),
        ("k_cap_max", ctypes.c_int32),
        ("num_wg", ctypes.c_int32),
        ("row_depth", ctypes.c_int32),
    ]


class RBRPError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


_lib = None

_c = ctypes
_vp, _i64, _i32, _u64, _dbl, _sz = (_c.c_void_p, _c.c_int64, _c.c_int32, _c.c_uint64,
                                    _c.c_double, _c.c_size_t)

# name -> (restype, argtypes); the exported C ABI
SIGNATURES = {
    "rbrp_default_options": (None, [_c.POINTER(rbrp_options)]),
    "rbrp_workspace_size": (_sz, [_c.c_int, _i64, _i64, _i32, _c.POINTER(rbrp_options)]),
    "rbrp_id": (_c.c_int, [_vp, _c.c_int, _i64, _i64, _i64, _dbl, _i32, _u64,
                           _c.POINTER(rbrp_options), _vp, _c.POINTER(_i64), _vp, _i64,
                           _c.POINTER(rbrp_stats), _vp, _sz, _vp]),
    "rbrp_status_string": (_c.c_char_p, [_c.c_int]),
    "rbrp_err_bound_increment": (_dbl, [_i32, _i32, _dbl, _dbl]),
    "rbrp_row_norms_workspace_size": (_sz, [_i64]),
    "rbrp_row_norms": (_c.c_int, [_vp, _c.c_int, _i64, _i64, _i64, _vp,
                                  _c.POINTER(_dbl), _c.POINTER(_dbl), _vp, _sz, _vp]),
    "rbrp_sample_workspace_size": (_sz, [_i64]),
    "rbrp_sample_block": (_c.c_int, [_vp, _vp, _i64, _i32, _u64, _u64, _u64, _vp,
                                     _c.POINTER(_i32), _vp, _sz, _vp]),
    "rbrp_block_cpqr_workspace_size": (_sz, [_i64, _i32]),
    "rbrp_block_cpqr": (_c.c_int, [_vp, _i64, _i32, _i64, _dbl, _vp, _vp, _vp, _i64,
                                   _c.POINTER(_i32), _vp, _sz, _vp]),
    "rbrp_sketchy_workspace_size": (_sz, [_c.c_int, _i64, _i64, _i32, _i32]),
    "rbrp_sketchy_id": (_c.c_int, [_vp, _c.c_int, _i64, _i64, _i64, _i32, _i32, _vp, _i64,
                                   _vp, _vp, _i64, _vp, _sz, _vp]),
    "rbrp_batch_workspace_size": (_sz, [_c.c_int, _c.POINTER(rbrp_batch_shape)]),
    "rbrp_id_batched": (_c.c_int, [_vp, _vp, _i32, _c.c_int, _dbl, _u64,
                                   _c.POINTER(rbrp_options), _c.POINTER(rbrp_batch_shape),
                                   _vp, _vp, _vp, _vp, _sz, _vp]),
    "rbrp_id_batched_noalloc": (_c.c_int, [_vp, _vp, _i32, _c.c_int, _dbl, _u64,
                                           _c.POINTER(rbrp_options),
                                           _c.POINTER(rbrp_batch_shape), _vp, _vp, _vp, _vp]),
    "rbrp_batch_autotune": (_c.c_int, [_c.POINTER(rbrp_batch_desc), _vp, _i32, _c.c_int,
                                       _dbl, _u64, _c.POINTER(rbrp_options),
                                       _c.POINTER(rbrp_batch_shape), _vp, _vp, _vp, _vp,
                                       _vp, _sz, _vp, _c.POINTER(_i32)]),
}


def lib():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"RBRP HIP library not built: {LIB_PATH} is missing "
                "(run python -m paper_2309_16002_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_string(status):
    return lib().rbrp_status_string(int(status)).decode()


def _torch():
    import torch
    return torch


def _stream_ptr(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float32:
        return RBRP_F32
    if t.dtype == torch.float64:
        return RBRP_F64
    raise TypeError(f"unsupported dtype {t.dtype}: use float32 or float64")


def _ld(t):
    """Leading dimension of a row-major 2-D tensor (a single row may carry any
    row stride)."""
    return t.stride(0) if t.shape[0] > 1 else t.shape[1]


def _check_matrix(X):
    if not X.is_cuda:
        raise ValueError("X must be a GPU tensor")
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a 2-D row-major tensor (unit column stride)")


W_METHODS = {"substitution": 0, "svd": 1}


def make_options(k_max=0, tau_b=None, fixed_rank=False, greedy=False, precision="native",
                 theta=0.0, w_refine=-1, profile=False, trim=False, replay_d=None,
                 w_method="substitution", w_clip=0.0):
    o = rbrp_options()
    lib().rbrp_default_options(ctypes.byref(o))
    o.tau_b = -1.0 if tau_b is None else float(tau_b)
    o.k_max = int(k_max)
    o.fixed_rank = int(bool(fixed_rank))
    o.greedy = int(bool(greedy))
    o.precision = PRECISIONS[precision]
    o.theta = float(theta)
    o.w_refine = int(w_refine)
    o.profile = 2 if profile == "deflate" else int(bool(profile))
    o.trim = int(bool(trim))
    o.w_method = W_METHODS[w_method]
    o.w_clip = float(w_clip)
    if replay_d is not None:
        # test hook: [blocks, m] FP64 device tensor of the norms each block
        # samples from (the caller keeps it alive for the call)
        if replay_d.dtype != _torch().float64 or not replay_d.is_cuda or replay_d.dim() != 2 \
                or not replay_d.is_contiguous():
            raise ValueError("replay_d must be a contiguous [blocks, m] float64 GPU tensor")
        o.replay_d = replay_d.data_ptr()
        o.replay_blocks = int(replay_d.shape[0])
    return o


@dataclass
class IDResult:
    S: object            # int64 tensor [k], selection order
    k: int
    W: object            # float64 tensor [m, k] or None
    status: int
    blocks: int
    blocks_split: int
    bprime: list
    resid_tracked: float
    norm_x: float
    profile: dict = None
    err_bound: float = 0.0       # bound on the rounding in the tracked residual
    blocks_native: int = 0       # BF16 form: blocks deflated with the FP32 product
    blocks_bf16_stored: int = 0  # BF16 form: blocks whose residual was stored in BF16
    w_rank: int = 0              # singular values of L_1 kept (w_method="svd"), else k


def workspace_size(m, n, b, dtype="f32", **opts):
    o = make_options(**opts)
    dt = RBRP_F32 if dtype in ("f32", "float32") else RBRP_F64
    return int(lib().rbrp_workspace_size(dt, int(m), int(n), int(b), ctypes.byref(o)))


def rbrp_id(X, eps, b, seed=0, *, want_w=True, workspace=None, out_S=None, out_W=None,
            **opts):
    """Row ID X ~= W X[S] by RBRP (Algorithm 2, then Algorithm 3).

    ``workspace``, ``out_S`` (int64 [k_max]) and ``out_W`` (float64 [m, k_max],
    row-major) may be passed in to reuse device buffers across calls."""
    torch = _torch()
    _check_matrix(X)
    L = lib()
    m, n = X.shape
    dt = _dtype_code(X)
    o = make_options(**opts)
    ws_bytes = L.rbrp_workspace_size(dt, m, n, int(b), ctypes.byref(o))
    if ws_bytes == 0:
        raise RBRPError(RBRP_E_INVALID, "rbrp_workspace_size")
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=X.device)
    k_max = o.k_max if o.k_max > 0 else min(m, n)
    S = out_S if out_S is not None else torch.empty(k_max, dtype=torch.int64, device=X.device)
    if S.numel() < k_max or S.dtype != torch.int64 or not S.is_contiguous():
        raise ValueError("out_S must be a contiguous int64 tensor of at least k_max entries")
    W = None
    if want_w:
        W = out_W if out_W is not None else torch.empty((m, k_max), dtype=torch.float64,
                                                        device=X.device)
        if (W.dtype != torch.float64 or W.dim() != 2 or W.shape[0] != m
                or W.shape[1] < k_max or W.stride(1) != 1):
            raise ValueError("out_W must be a row-major float64 [m, >= k_max] tensor")
    k = ctypes.c_int64(0)
    st = rbrp_stats()
    status = L.rbrp_id(_ptr(X), dt, m, n, _ld(X), float(eps), int(b), int(seed),
                       ctypes.byref(o), _ptr(S), ctypes.byref(k), _ptr(W),
                       W.stride(0) if W is not None else k_max,
                       ctypes.byref(st), _ptr(workspace), ws_bytes, _stream_ptr(X.device))
    if status not in (RBRP_OK, RBRP_E_CAPACITY):
        raise RBRPError(status, "rbrp_id")
    kk = int(k.value)
    nb = min(st.blocks, 256)
    prof = None
    if o.profile:
        prof = dict(ms_init=st.ms_init, ms_select=st.ms_select, ms_filter=st.ms_filter,
                    ms_deflate=st.ms_deflate, ms_interp=st.ms_interp,
                    deflate_flops=st.deflate_flops, deflate_launches=st.deflate_launches,
                    deflate_bytes=st.deflate_bytes)
    return IDResult(S[:kk], kk, W[:, :kk] if W is not None else None, status, st.blocks,
                    st.blocks_split, [int(x) for x in st.bprime[:nb]], st.resid_tracked,
                    st.norm_x_fro, prof, st.err_bound, st.blocks_native,
                    st.blocks_bf16_stored, st.w_rank)


DEFLATE_MODES = {"f64": 0, "f32": 1, "bf16x3": 2, "bf16": 3, "bf16_stored": 4}


def sketchy_id(X, Omega, k, *, want_w=True, workspace=None):
    """Sketchy pivoting (LU with partial pivoting on Y = X Omega) and the
    oversampled sketchy interpolation matrix (Algorithm 4).  Omega: FP64
    [n, l] GPU tensor (the caller's embedding).  Returns (S [k] int64, W
    [m, k] float64 or None)."""
    torch = _torch()
    _check_matrix(X)
    L = lib()
    m, n = X.shape
    if (Omega.dtype != torch.float64 or not Omega.is_cuda or Omega.dim() != 2
            or Omega.shape[0] != n or Omega.stride(1) != 1):
        raise ValueError("Omega must be a row-major float64 [n, l] GPU tensor")
    l = Omega.shape[1]
    dt = _dtype_code(X)
    ws_bytes = L.rbrp_sketchy_workspace_size(dt, m, n, int(k), int(l))
    if ws_bytes == 0:
        raise RBRPError(RBRP_E_INVALID, "rbrp_sketchy_workspace_size")
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=X.device)
    S = torch.empty(int(k), dtype=torch.int64, device=X.device)
    W = torch.empty((m, int(k)), dtype=torch.float64, device=X.device) if want_w else None
    status = L.rbrp_sketchy_id(_ptr(X), dt, m, n, _ld(X), int(k), int(l), _ptr(Omega),
                               _ld(Omega), _ptr(S), _ptr(W), int(k), _ptr(workspace), ws_bytes,
                               _stream_ptr(X.device))
    if status != RBRP_OK:
        raise RBRPError(status, "rbrp_sketchy_id")
    return S, W


def err_bound_increment(mode, bprime, r_prev_sq, r_new_sq):
    """Variance increment of the rounding bound after one deflated block
    (host arithmetic of the library; see rbrp_err_bound_increment)."""
    code = DEFLATE_MODES[mode] if isinstance(mode, str) else int(mode)
    return float(lib().rbrp_err_bound_increment(code, int(bprime), float(r_prev_sq),
                                                float(r_new_sq)))


def row_norms(X):
    """d_i = ||x_i||^2 in FP64 (Alg. 2 initialisation); returns (d, sum, max)."""
    torch = _torch()
    _check_matrix(X)
    L = lib()
    m, n = X.shape
    d = torch.empty(m, dtype=torch.float64, device=X.device)
    ws_bytes = L.rbrp_row_norms_workspace_size(m)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=X.device)
    s, mx = ctypes.c_double(0), ctypes.c_double(0)
    status = L.rbrp_row_norms(_ptr(X), _dtype_code(X), m, n, _ld(X), _ptr(d),
                              ctypes.byref(s), ctypes.byref(mx), _ptr(ws), ws_bytes,
                              _stream_ptr(X.device))
    if status != RBRP_OK:
        raise RBRPError(status, "rbrp_row_norms")
    return d, s.value, mx.value


def sample_block(d, excluded, b, seed, t, ident=0):
    """One block of Alg. 2's sampler; returns an int64 tensor of indices."""
    torch = _torch()
    L = lib()
    if d.dtype != torch.float64 or not d.is_cuda or d.dim() != 1:
        raise ValueError("d must be a 1-D float64 GPU tensor")
    d = d.contiguous()
    m = d.shape[0]
    ex = None
    if excluded is not None:
        ex = excluded.to(device=d.device, dtype=torch.uint8).contiguous()
    idx = torch.empty(max(int(b), 1), dtype=torch.int64, device=d.device)
    ws_bytes = L.rbrp_sample_workspace_size(m)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=d.device)
    nout = ctypes.c_int32(0)
    status = L.rbrp_sample_block(_ptr(d), _ptr(ex), m, int(b), int(seed), int(t), int(ident),
                                 _ptr(idx), ctypes.byref(nout), _ptr(ws), ws_bytes,
                                 _stream_ptr(d.device))
    if status != RBRP_OK:
        raise RBRPError(status, "rbrp_sample_block")
    return idx[: nout.value]


def block_cpqr(Vt, tau_b):
    """Robust blockwise filter on one block (rows of Vt = columns of V).

    Returns (piv int32 [nb], R float64 [nb, nb], Qt float64 [b', n], b')."""
    torch = _torch()
    L = lib()
    if Vt.dtype != torch.float64 or not Vt.is_cuda or Vt.dim() != 2 or Vt.stride(1) != 1:
        raise ValueError("Vt must be a 2-D row-major float64 GPU tensor")
    nb, n = Vt.shape
    piv = torch.empty(nb, dtype=torch.int32, device=Vt.device)
    R = torch.empty((nb, nb), dtype=torch.float64, device=Vt.device)
    Qt = torch.zeros((nb, n), dtype=torch.float64, device=Vt.device)
    ws_bytes = L.rbrp_block_cpqr_workspace_size(n, nb)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=Vt.device)
    bp = ctypes.c_int32(0)
    status = L.rbrp_block_cpqr(_ptr(Vt), n, nb, _ld(Vt), float(tau_b), _ptr(piv), _ptr(R),
                               _ptr(Qt), n, ctypes.byref(bp), _ptr(ws), ws_bytes,
                               _stream_ptr(Vt.device))
    if status != RBRP_OK:
        raise RBRPError(status, "rbrp_block_cpqr")
    return piv, R, Qt[: bp.value], int(bp.value)


class BatchPlan:
    """Device buffers of one batch of independent IDs (rbrp_id_batched).

    Built once per set of input matrices; a launch only passes pointers, so
    it can be captured in a graph.  Outputs are packed: ``S_all`` holds
    k_cap_i entries per ID, ``W_all`` an m_i x k_cap_i block per ID."""

    def __init__(self, Xs, b=16, k_caps=None, want_w=True, num_wg=0):
        torch = _torch()
        if not Xs:
            raise ValueError("empty batch")
        dev = Xs[0].device
        dt = _dtype_code(Xs[0])
        for X in Xs:
            _check_matrix(X)
            if _dtype_code(X) != dt or X.device != dev:
                raise ValueError("all matrices of a batch share dtype and device")
        self.Xs = list(Xs)
        self.count = len(Xs)
        self.dtype = dt
        self.device = dev
        ms = [int(X.shape[0]) for X in Xs]
        ns = [int(X.shape[1]) for X in Xs]
        ks = [min(m, n) for m, n in zip(ms, ns)] if k_caps is None else [int(k) for k in k_caps]
        self.ms, self.ns, self.ks = ms, ns, ks
        self.s_off = [0]
        for k in ks:
            self.s_off.append(self.s_off[-1] + k)
        self.w_off = [0]
        for m, k in zip(ms, ks):
            self.w_off.append(self.w_off[-1] + m * k)
        self.S_all = torch.empty(max(self.s_off[-1], 1), dtype=torch.int64, device=dev)
        self.W_all = (torch.empty(max(self.w_off[-1], 1), dtype=torch.float64, device=dev)
                      if want_w else None)
        self.k_out = torch.zeros(self.count, dtype=torch.int32, device=dev)
        self.status_out = torch.zeros(self.count, dtype=torch.int32, device=dev)
        self.resid_out = torch.zeros(self.count, dtype=torch.float64, device=dev)
        self.order = torch.arange(self.count, dtype=torch.int32, device=dev)
        self.shape = rbrp_batch_shape()
        self.shape.m_max = max(ms)
        self.shape.n_max = max(ns)
        self.shape.b_max = 32
        self.shape.k_cap_max = max(ks)
        self.shape.num_wg = int(num_wg)
        self.descs_host = (rbrp_batch_desc * self.count)()
        for i, X in enumerate(Xs):
            d = self.descs_host[i]
            d.X = X.data_ptr()
            d.m, d.n, d.ldx = ms[i], ns[i], _ld(X)
            d.S = self.S_all.data_ptr() + 8 * self.s_off[i]
            d.W = (self.W_all.data_ptr() + 8 * self.w_off[i]) if want_w else None
            d.ldw = ks[i]
            d.k_cap = ks[i]
            d.b = int(b)
        raw = bytes(self.descs_host)
        self.descs = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
        self._alloc_workspace()

    def _alloc_workspace(self, num_wg=None):
        torch = _torch()
        sh = rbrp_batch_shape.from_buffer_copy(self.shape)
        if num_wg is not None:
            sh.num_wg = num_wg
        nbytes = int(lib().rbrp_batch_workspace_size(self.dtype, ctypes.byref(sh)))
        if nbytes == 0:
            raise RBRPError(RBRP_E_INVALID, "rbrp_batch_workspace_size")
        if getattr(self, "workspace", None) is None or self.workspace.numel() < nbytes:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    def result(self, i):
        """(S, k, W, status, tracked residual) of ID i (synchronises)."""
        k = int(self.k_out[i].item())
        S = self.S_all[self.s_off[i]:self.s_off[i] + k]
        W = None
        if self.W_all is not None:
            W = self.W_all[self.w_off[i]:self.w_off[i + 1]].view(self.ms[i], self.ks[i])[:, :k]
        return S, k, W, int(self.status_out[i].item()), float(self.resid_out[i].item())


def rbrp_id_batched(plan, eps, seed=0, stream=None, **opts):
    """Launch all IDs of ``plan`` (no synchronisation; outputs in the plan)."""
    o = make_options(**opts)
    st = stream if stream is not None else _stream_ptr(plan.device)
    status = lib().rbrp_id_batched(_ptr(plan.descs), _ptr(plan.order), plan.count,
                                   plan.dtype, float(eps), int(seed), ctypes.byref(o),
                                   ctypes.byref(plan.shape), _ptr(plan.k_out),
                                   _ptr(plan.status_out), _ptr(plan.resid_out),
                                   _ptr(plan.workspace), plan.workspace.numel(), st)
    if status != RBRP_OK:
        raise RBRPError(status, "rbrp_id_batched")
    return plan


def rbrp_id_batched_noalloc(plan, eps, seed=0, stream=None, **opts):
    """Launch all IDs of ``plan`` on the library's static scratch array instead
    of ``plan.workspace`` (no synchronisation, no allocation; outputs in the
    plan).  Calls that overlap on one GPU race on that array."""
    o = make_options(**opts)
    st = stream if stream is not None else _stream_ptr(plan.device)
    status = lib().rbrp_id_batched_noalloc(_ptr(plan.descs), _ptr(plan.order), plan.count,
                                           plan.dtype, float(eps), int(seed), ctypes.byref(o),
                                           ctypes.byref(plan.shape), _ptr(plan.k_out),
                                           _ptr(plan.status_out), _ptr(plan.resid_out), st)
    if status != RBRP_OK:
        raise RBRPError(status, "rbrp_id_batched_noalloc")
    return plan


def batch_autotune(plan, eps, seed=0, **opts):
    """Tune block size per size class and the persistent grid; returns the
    chosen block size per class (n <= 64, <= 128, > 128)."""
    o = make_options(**opts)
    plan._alloc_workspace(num_wg=768)
    bcls = (ctypes.c_int32 * 3)()
    status = lib().rbrp_batch_autotune(plan.descs_host, _ptr(plan.descs), plan.count,
                                       plan.dtype, float(eps), int(seed), ctypes.byref(o),
                                       ctypes.byref(plan.shape), _ptr(plan.order),
                                       _ptr(plan.k_out), _ptr(plan.status_out),
                                       _ptr(plan.resid_out), _ptr(plan.workspace),
                                       plan.workspace.numel(), _stream_ptr(plan.device),
                                       bcls)
    if status != RBRP_OK:
        raise RBRPError(status, "rbrp_batch_autotune")
    return [int(x) for x in bcls]
