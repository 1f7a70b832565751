#!/usr/bin/env python3
"""Benchmark: time to an eps-accurate RBRP interpolative decomposition on one
MI355X, reported as rows per second.

One step is one complete decomposition (``rbrp_id``): initial norms, every
sampled block (sampling, robust blockwise filter, basis update, deflation)
until the tracked residual meets eps, and the interpolation matrix W.  The
input matrix is resident in HBM before the timed region starts; outputs stay
on the device.  Each step uses a different sampling seed (0, 1, 2, ...).

Workload (default): the precision-form workload, X = U diag(s) V^T with
Haar factors and s_i = i^-1.5, 200000 x 2048 FP32, eps = 1e-4, block size
b = 128: FP32 ("plain") deflation products for ``value``, the BF16 form
beside it.  Other workloads with ``--workload``.

A step is eps-accurate when the library returned OK, which it does only when
the tracked residual plus its rounding bound E met eps (rho + E <= eps); the
last step's interpolation error ||X - W X_S||_F / ||X||_F is also recomputed
in FP64 (untimed) and must meet eps.

The JSON line carries:
  roofline      the fused deflation kernel (the O(m n k) part, R <- R - (R Q') Q'^T
                with the row norms): its arithmetic intensity is b'/2 flop per
                byte of FP32 residual traffic, so it is bound by the FP32 MFMA
                peak when b' > 39 (the default workload keeps b' ~ 128) and by
                HBM below that (the GMM workload, b' ~ 28); achieved =
                algorithmic flops 4 m n b' (or bytes: R read + written, the new
                L columns, d) per launch over the kernel's average duration,
                timed with HIP events that the library records on its own
                stream inside the timed region.  Both figures are in
                roofline["mfma"] and roofline["hbm"];
  bf16_form     the same workload with the BF16 precision form (deflation
                products on BF16 MFMA, FP32 accumulation), timed the same way:
                the metric's "BF16-MFMA vs FP32 plain" comparison;
  cpu_baseline  the CPU FP64 oracle (literal Algorithm 2 + Algorithm 3) on the
                same matrix, median of a few runs on the host's cores.
"""

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("time to eps-accurate ID (rows/sec) BF16-MFMA vs FP32 plain at eps; "
          "% MFMA peak")
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "f64": 78.6}
HBM_GBS = 8000.0

WORKLOADS = {
    "adversarial_gmm_fp32": dict(m=100000, n=1000, eps=1e-3, b=64, dtype="f32"),
    "svd_geometric_fp64": dict(m=2000, n=500, eps=1e-2, b=16, dtype="f64"),
    "svd_power_bf16": dict(m=200000, n=2048, eps=1e-4, b=128, dtype="f32"),
    # eps-rank at 1e-3 is close to n: run to the fixed rank k = 2048; the CPU
    # oracle runs on the first 4000 rows
    "random_features_large": dict(m=1000000, n=4096, eps=1e-3, b=256, dtype="f32",
                                  k_max=2048, fixed_rank=True, cpu_rows=4000),
    "kernel_blocks_batched": dict(count=4096, eps=1e-6, dtype="f32"),
}
RIDGE = {d: PEAK_TFLOPS[d] * 1e12 / (HBM_GBS * 1e9) for d in PEAK_TFLOPS}


def _kernel_sha():
    path = os.path.join(ROOT, "paper_2309_16002_amd", "csrc", "k_deflate.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(workload, form="fp32"):
    """HBM bytes per deflation launch (FETCH_SIZE + WRITE_SIZE, calibrated
    against a copy kernel) from the committed rocprofv3 counter summary of
    this workload, for the FP32 plain form or the BF16 form's mix of
    launches; None unless it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"deflate_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha") != _kernel_sha():
        return None
    return (rec.get(form) or {}).get("bytes_per_launch")


def make_input(name):
    from workloads import config_matrix
    return config_matrix(name)


def cpu_baseline(X, cfg, budget_s, max_repeats):
    """The oracle as it stands, on the host's cores: whole decompositions of
    the same matrix (seeds 0, 1, ...) until about ``budget_s`` seconds of work
    (at most ``max_repeats``); the median run time gives rows/s."""
    import numpy as np
    from oracle import rbrp as oracle_rbrp, w_from_l
    try:
        from threadpoolctl import threadpool_info
        cores = max((p.get("num_threads", 1) for p in threadpool_info()
                     if p.get("user_api") == "blas"), default=os.cpu_count())
    except Exception:  # pragma: no cover - threadpoolctl is optional
        cores = os.cpu_count()
    rows = cfg.get("cpu_rows")
    X64 = np.asarray(X[:rows] if rows else X, dtype=np.float64)
    kw = {}
    if cfg.get("fixed_rank"):
        kw = dict(k_max=min(cfg["k_max"], min(X64.shape)), fixed_rank=True)
    times = []
    k = None
    while len(times) < max_repeats and sum(times) < budget_s:
        t0 = time.perf_counter()
        res = oracle_rbrp(X64, cfg["eps"], cfg["b"], seed=len(times), form="A", **kw)
        w_from_l(res.L, res.S)
        times.append(time.perf_counter() - t0)
        k = res.k
    t = statistics.median(times)
    m = X64.shape[0]
    return {"value": m / t, "unit": "rows/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"{'first rows of the ' if rows else 'full '}workload "
                       f"{X64.shape[0]}x{X64.shape[1]} (FP32 input promoted "
                       f"to FP64), literal Algorithm 2 + Algorithm 3, {len(times)} runs "
                       f"(seeds 0..{len(times) - 1}, {sum(times):.1f} s of work), median "
                       f"{t:.3f} s per run, k={k}")}


def bench_batched(args, cfg):
    """The batched form: all IDs of the batch in one persistent launch,
    captured once in a HIP graph and replayed; a step is one replay."""
    import numpy as np
    import torch
    import paper_2309_16002_amd as rb
    from workloads import kernel_blocks
    print("[bench] generating kernel_blocks_batched", file=sys.stderr, flush=True)
    Xs = kernel_blocks(count=cfg["count"], seed=1004)
    dev = torch.device("cuda:0")
    Xg = [torch.from_numpy(X).to(dev) for X in Xs]
    plan = rb.BatchPlan(Xg, b=16)
    eps = cfg["eps"]
    t0 = time.perf_counter()
    bcls = rb.batch_autotune(plan, eps, 0)
    tune_s = time.perf_counter() - t0
    depth = [(plan.shape.row_depth >> (4 * c)) & 15 for c in range(3)]
    print(f"[bench] autotuned b per class {bcls}, row-load depth per class {depth}, "
          f"{plan.shape.num_wg} workgroups ({tune_s:.1f} s)", file=sys.stderr, flush=True)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            rb.rbrp_id_batched(plan, eps, 0)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    rows = sum(plan.ms)
    ms_step = 1e3 * total / args.steps
    # untimed checks of every ID of the last replay
    status = plan.status_out.cpu().numpy()
    ks = plan.k_out.cpu().numpy()
    resid = plan.resid_out.cpu().numpy()
    worst = 0.0
    for i in range(0, plan.count, max(1, plan.count // 256)):
        S, k, W, st, _ = plan.result(i)
        X64 = torch.from_numpy(Xs[i]).to(dev).double()
        E = X64 - W @ X64[S]
        worst = max(worst, (torch.linalg.norm(E) / torch.linalg.norm(X64)).item())
    accurate = bool((status == 0).all()) and worst <= eps * (1 + 1e-6) + 3e-7
    # algorithmic HBM bytes: X read once, W written once
    nbytes = sum(m * n * 4 for m, n in zip(plan.ms, plan.ns)) + \
        sum(int(m) * int(k) * 8 for m, k in zip(plan.ms, ks))
    gbs = nbytes / (ms_step * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": rows / (ms_step * 1e-3), "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "kernel_blocks_batched", "count": plan.count,
                   "rows_total": rows, "eps": eps, "b_per_class": bcls,
                   "row_depth_per_class": depth,
                   "num_wg": plan.shape.num_wg, "launch": "one persistent kernel in a HIP graph",
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_GBS, 4), "traffic": None,
                     "kernel": "k_rbrp_batched (latency-bound; algorithmic bytes: X read, W "
                               "written)"},
        "eps_accurate": accurate, "max_rel_error_sampled": worst,
        "k_mean": float(ks.mean()), "k_max": int(ks.max()),
        "max_tracked_residual": float(resid.max()),
    }
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        from oracle import rbrp as oracle_rbrp, w_from_l
        try:
            from threadpoolctl import threadpool_info
            cores = max((p.get("num_threads", 1) for p in threadpool_info()
                         if p.get("user_api") == "blas"), default=os.cpu_count())
        except Exception:  # pragma: no cover
            cores = os.cpu_count()
        done_rows, t_cpu, i = 0, 0.0, 0
        while t_cpu < args.cpu_budget and i < plan.count:
            X64 = Xs[i].astype(np.float64)
            t1 = time.perf_counter()
            res = oracle_rbrp(X64, eps, 16, 0, form="A", ident=i)
            w_from_l(res.L, res.S)
            t_cpu += time.perf_counter() - t1
            done_rows += X64.shape[0]
            i += 1
        line["cpu_baseline"] = {
            "value": done_rows / t_cpu, "unit": "rows/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"the first {i} IDs of the batch ({done_rows} rows, b=16), one after "
                      f"another, {t_cpu:.1f} s"}
    print(json.dumps(line), flush=True)


def bench_sketchy(args, cfg, X):
    """Sketchy pivoting (LU with partial pivoting on Y = X Omega) and the
    oversampled sketchy ID (Algorithm 4) at a fixed rank k, l = 3k: the
    comparison method of the paper's Table 3.  A step is one rbrp_sketchy_id
    call; Omega is drawn once (Gaussian, seeded) and stays resident."""
    import numpy as np
    import torch
    import paper_2309_16002_amd as rb
    dev = torch.device("cuda:0")
    m, n = X.shape
    k = args.sketchy
    l = args.sketch_l or 3 * k
    Xg = torch.from_numpy(X).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    Omega = torch.randn((n, l), dtype=torch.float64, device=dev, generator=gen)
    for _ in range(args.warmup):
        S, W = rb.sketchy_id(Xg, Omega, k)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[2 * i].record()
        S, W = rb.sketchy_id(Xg, Omega, k)
        ev[2 * i + 1].record()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ms_call = statistics.mean(ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(args.steps))
    X64 = Xg.double()
    err = float(torch.linalg.norm(X64 - W @ X64[S]) / torch.linalg.norm(X64))
    # executed FP64 flops: the sketch 2 m n l, the elimination about m k^2,
    # the OSID product 2 m l k (the QR of the l x k skeleton sketch is small)
    flops = 2.0 * m * n * l + 1.0 * m * k * k + 2.0 * m * l * k
    tfl = flops / (ms_call * 1e-3) / 1e12
    line = {
        "metric": METRIC, "value": m * args.steps / total, "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "method": "SkLUPP-OSID",
                   "k": k, "l": l, "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": round(tfl, 3), "peak": PEAK_TFLOPS["f64"],
                     "unit": "TFLOP/s", "frac": round(tfl / PEAK_TFLOPS["f64"], 4),
                     "traffic": None,
                     "kernel": "whole rbrp_sketchy_id call (FP64 sketch, elimination, OSID)"},
        "rel_error_last_step": err,
    }
    if not args.no_cpu_baseline:
        from oracle.sketchy import sketchy_id as oracle_sketchy
        Om = Omega.cpu().numpy()
        X64h = np.asarray(X, dtype=np.float64)
        times = []
        while len(times) < args.cpu_repeats and sum(times) < args.cpu_budget:
            t1 = time.perf_counter()
            oracle_sketchy(X64h, Om, k)
            times.append(time.perf_counter() - t1)
        t = statistics.median(times)
        line["cpu_baseline"] = {"value": m / t, "unit": "rows/s", "cores": os.cpu_count(),
                                "kind": "oracle",
                                "sample": f"full workload, {len(times)} runs, median {t:.3f} s"}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="svd_power_bf16", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=10.0, metavar="SECONDS",
                    help="CPU oracle baseline: seconds of oracle work to time")
    ap.add_argument("--cpu-repeats", type=int, default=31, help="at most this many oracle runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the BF16 precision-form leg")
    ap.add_argument("--block", type=int, default=0, metavar="B",
                    help="override the workload's block size b (b = 1 is sequential random "
                         "pivoting, Algorithm 1: the matrix-vector baseline)")
    ap.add_argument("--greedy", action="store_true",
                    help="blockwise greedy pivoting (the b largest residual norms, Remark 4.3) "
                         "instead of sampling; with --block 1 this is column-pivoted QR")
    ap.add_argument("--trim", action="store_true",
                    help="rank trimming: cut k to the shortest prefix of the selection "
                         "that meets eps (an option of rbrp_id; off in the default line)")
    ap.add_argument("--fixed-rank", type=int, default=0, metavar="K",
                    help="run to exactly K skeletons (Alg. 2's 'or k' rule; the protocol of the "
                         "paper's Table 3) instead of to eps")
    ap.add_argument("--to-eps", action="store_true",
                    help="run to the workload's eps with k_max = min(m, n) even where the "
                         "workload is defined at a fixed rank (random_features_large)")
    ap.add_argument("--sketchy", type=int, default=0, metavar="K",
                    help="time sketchy pivoting with LU + the oversampled sketchy ID (Alg. 4) "
                         "at rank K instead of RBRP")
    ap.add_argument("--sketch-l", type=int, default=0, metavar="L",
                    help="sketch size for --sketchy (default 3K)")
    ap.add_argument("--w-method", default="substitution", choices=["substitution", "svd"],
                    help="interpolation matrix: blocked substitution with one refinement "
                         "step (Alg. 3, the default) or the truncated-SVD pseudo-inverse of "
                         "L_1 (Remark 5.2)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device-to-device copy of MB megabytes (the "
                         "reference for HBM byte counters) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} (WORLD_SIZE {world}) is not "
              "supported: every decomposition runs on a single MI355X.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2309_16002_amd as rb

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        n_el = args.copy_calibration * 1000000 // 4
        src = torch.ones(n_el, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n_el * 4}))
        return
    rb.lib()
    cfg = dict(WORKLOADS[args.workload])
    if args.block:
        cfg["b"] = args.block
    if args.workload == "kernel_blocks_batched":
        bench_batched(args, cfg)
        return
    if args.fixed_rank:
        cfg["k_max"] = args.fixed_rank
        cfg["fixed_rank"] = True
    if args.to_eps:
        cfg.pop("k_max", None)
        cfg["fixed_rank"] = False
    if args.sketchy:
        print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
        bench_sketchy(args, cfg, make_input(args.workload))
        return
    dev = torch.device("cuda:0")
    print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
    X = make_input(args.workload)
    m, n = X.shape
    Xg = torch.from_numpy(X).to(dev)
    k_max = cfg.get("k_max") or min(m, n)
    fixed = bool(cfg.get("fixed_rank"))
    need = max(rb.workspace_size(m, n, cfg["b"], cfg["dtype"], precision=p, k_max=k_max)
               for p in (("native", "bf16") if cfg["dtype"] == "f32" else ("native",)))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    S_buf = torch.empty(k_max, dtype=torch.int64, device=dev)
    W_buf = torch.empty((m, k_max), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def run_form(precision, steps, warmup):
        """Time `steps` decompositions in one precision form; returns the
        per-step results, the wall time, the last step's FP64 error and the
        phase times of one extra untimed step.  Inside the timed loop only
        the deflation launches are bracketed by HIP events (their durations
        give the roofline figures)."""
        def step(seed, profile="deflate"):
            return rb.rbrp_id(Xg, cfg["eps"], cfg["b"], seed, workspace=ws, out_S=S_buf,
                              out_W=W_buf, precision=precision, profile=profile,
                              k_max=k_max, fixed_rank=fixed, trim=args.trim,
                              greedy=args.greedy, w_method=args.w_method)
        for i in range(warmup):
            step(1000 + i)
            print(f"[bench] {precision} warmup {i + 1}/{warmup} done", file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        results = []
        t0 = time.perf_counter()
        for i in range(steps):
            results.append(step(i))
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        print(f"[bench] {precision}: timed {steps} steps in {total:.3f} s", file=sys.stderr,
              flush=True)
        # untimed check that the result met eps: ||X - W X_S||_F <= eps ||X||_F
        # in FP64 for the last step (its outputs are still in the buffers),
        # in row chunks
        last = results[-1]
        XS = Xg[last.S].double()
        e2 = x2 = 0.0
        for r0 in range(0, m, 100000):
            Xc = Xg[r0:r0 + 100000].double()
            Ec = Xc - last.W[r0:r0 + 100000] @ XS
            e2 += float(torch.sum(Ec * Ec))
            x2 += float(torch.sum(Xc * Xc))
            del Xc, Ec
        err = (e2 / x2) ** 0.5
        del XS
        phased = step(0, profile=True)
        phases = {key: round(phased.profile[key], 4)
                  for key in ("ms_init", "ms_select", "ms_filter", "ms_deflate", "ms_interp")}
        return results, total, err, phases

    def deflation_roofline(results, dtype):
        """Algorithmic flops and bytes of the deflation launches (the library
        counts them: 4 m n b' flops per block; the residual read and written
        in its storage type, d, and the new columns of L) over their HIP-event
        durations."""
        flops = sum(r.profile["deflate_flops"] for r in results)
        ms_def = sum(r.profile["ms_deflate"] for r in results)
        launches = sum(r.profile["deflate_launches"] for r in results)
        nbytes = sum(r.profile["deflate_bytes"] for r in results)
        sec = ms_def * 1e-3
        gbs = nbytes / sec / 1e9 if sec > 0 else 0.0
        tfl = flops / sec / 1e12 if sec > 0 else 0.0
        ai = flops / nbytes if nbytes > 0 else 0.0
        mfma = {"achieved": round(tfl, 3), "peak": PEAK_TFLOPS[dtype], "unit": "TFLOP/s",
                "frac": round(tfl / PEAK_TFLOPS[dtype], 4)}
        hbm = {"achieved": round(gbs, 1), "peak": HBM_GBS, "unit": "GB/s",
               "frac": round(gbs / HBM_GBS, 4)}
        bound = "hbm" if ai < RIDGE[dtype] else "mfma"
        head = hbm if bound == "hbm" else mfma
        return dict(bound=bound, **head, launches=launches,
                    avg_launch_ms=round(ms_def / max(launches, 1), 4),
                    bytes_per_launch=nbytes / max(launches, 1),
                    flops_per_launch=flops / max(launches, 1),
                    arithmetic_intensity=round(ai, 2), ridge=round(RIDGE[dtype], 2),
                    mfma=mfma, hbm=hbm)

    def eps_accurate(results, err_last):
        """Every step stopped on rho + E <= eps (status OK) and the last
        step's recomputed FP64 error meets eps."""
        if fixed:
            return None
        return (all(r.status == 0 and r.resid_tracked + r.err_bound <= cfg["eps"]
                    for r in results) and err_last <= cfg["eps"])

    main_prec = "native"
    results, total, err_last, phases = run_form(main_prec, args.steps, args.warmup)
    accurate = eps_accurate(results, err_last)
    ms_per_step = 1e3 * total / args.steps
    value = m * args.steps / total
    dtype = cfg["dtype"]
    roofline = deflation_roofline(results, dtype)
    roofline["traffic"] = _traffic(args.workload)
    roofline["kernel"] = "k_deflate (P = R Q', R -= P Q'^T, row norms)"
    ks = [r.k for r in results]
    line = {
        "metric": METRIC, "value": value, "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "eps": cfg["eps"],
                   "b": cfg["b"], "tau_b": 1.0 / cfg["b"],
                   **({"fixed_rank": k_max} if fixed else {}),
                   **({"trim": True} if args.trim else {}),
                   **({"greedy": True} if args.greedy else {}),
                   **({"w_method": "truncated-SVD pseudo-inverse"}
                      if args.w_method == "svd" else {}),
                   "deflation": "fp64-mfma" if dtype == "f64" else "fp32-mfma (plain)",
                   "parallelism": "single-gpu"},
        "roofline": roofline,
        "eps_accurate": accurate, "rel_error_last_step": err_last,
        "max_tracked_residual": max(r.resid_tracked for r in results),
        "max_err_bound": max(r.err_bound for r in results),
        "k_median": statistics.median(ks), "k_range": [min(ks), max(ks)],
        "blocks_median": statistics.median(r.blocks for r in results),
        "phases_ms": phases,
    }
    if dtype == "f32" and not args.no_bf16:
        res16, tot16, err16, phases16 = run_form("bf16", args.steps, 1)
        v16 = m * args.steps / tot16
        rf16 = deflation_roofline(res16, "bf16")
        rf16["traffic"] = _traffic(args.workload, "bf16_form")
        line["bf16_form"] = {
            "value": v16, "unit": "rows/s", "ms_per_step": 1e3 * tot16 / args.steps,
            "speedup_vs_fp32_plain": v16 / value,
            "eps_accurate": eps_accurate(res16, err16),
            "rel_error_last_step": err16,
            "max_tracked_residual": max(r.resid_tracked for r in res16),
            "max_err_bound": max(r.err_bound for r in res16),
            "k_median": statistics.median(r.k for r in res16),
            "blocks_median": statistics.median(r.blocks for r in res16),
            "blocks_split_median": statistics.median(r.blocks_split for r in res16),
            "blocks_fp32_median": statistics.median(r.blocks_native for r in res16),
            "blocks_bf16_stored_median": statistics.median(r.blocks_bf16_stored for r in res16),
            "controller": "per block the cheapest of one BF16 product on a BF16-stored "
                          "residual, one BF16 product or split BF16 products on an FP32 "
                          "residual, and the FP32 product, that keeps the rounding bound "
                          "within eps/4",
            "deflation_roofline": rf16,
            "phases_ms": phases16,
        }
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(X, cfg, args.cpu_budget, args.cpu_repeats)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
