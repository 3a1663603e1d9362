"""Benchmark: Silhouette points/s on one MI355X.

One step = the whole hot path (per-cluster statistics, table finalisation, fused MFMA
GEMM+epilogue, reduction of S) over the resident synthetic workload, through the C ABI.

Default workload: blobs-50m-d128-k1000 (N=50,000,000, D=128, K=1000 Gaussian blobs), squared
Euclidean, X stored bf16, bf16 MFMA with fp32 accumulation.  The fp32 form (X stored fp32, fp32
MFMA) is timed beside it on the same points; |dS| between the two and against the whole FP64
oracle (every point, on the host) is reported, with the copy and GEMM rates this GPU reaches on
plain library work and the small workload's per-call latency.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2.5e15, "fp32": 157.3e12, "hbm": 8.0e12}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ["paper_2303_14102_amd/csrc/main_kernels.h", "paper_2303_14102_amd/csrc/main_bf16.hip",
                  "paper_2303_14102_amd/csrc/main_f32.hip", "paper_2303_14102_amd/csrc/stats.hip",
                  "paper_2303_14102_amd/csrc/main_screen.hip", "paper_2303_14102_amd/csrc/screen.hip"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, variant):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter summary, or None
    when it is missing, was taken on another form (variant: storage/metric/products, e.g.
    "bf16/sqeuclid/p2") or the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash() or t.get("variant") != variant:
        return None
    e = t.get("kernels", {}).get(f"{kernel}@{workload}")
    return None if e is None else e.get("hbm_bytes_per_launch")


def bench_kmeans(args, spec, X, col_scale, labels, dev):
    """One K-means (Lloyd) step per timed step: the means of the workload's labels, then every
    point's nearest mean, into a separate output so that every step does the same work."""
    import numpy as np
    import torch

    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    from paper_2303_14102_amd import workloads as wl
    lib = _lib.load()
    ws = sil.new_workspace(spec.n, spec.d, spec.k, "sqeuclid", X.dtype, 0, dev)
    out = torch.empty(spec.n, dtype=torch.int32, device=dev)
    inertia = torch.empty((), dtype=torch.float64, device=dev)
    dcode, stream, cs_ptr = sil._dtype_code(X), sil._stream(dev), sil._ptr(col_scale)
    kp = args.products if args.form == "bf16" else 0  # two products (folded centring) need bf16

    def step():
        rc = lib.silhouette_kmeans_step(sil._ptr(X), dcode, cs_ptr, sil._ptr(labels), spec.n, spec.d,
                                        spec.k, kp, 0, sil._ptr(out), sil._ptr(inertia), sil._ptr(ws),
                                        ws.numel(), stream)
        if rc:
            raise _lib.SilhouetteError(rc, "kmeans step")

    log(f"timing the K-means step ({args.form}): warmup {args.warmup}, steps {args.steps}")
    ms, phases, wall = timed_steps(step, args.steps, args.warmup, torch)
    _lib.check(sil.status(ws), "device status")
    moved = int((out != labels).sum().item())
    log(f"kmeans: {ms:.3f} ms/step, phases {['%.3f' % p for p in phases]}, inertia {inertia.item():.6e}, "
        f"moved {moved}")
    useful = 2.0 * spec.n * spec.d * spec.k
    t_main = phases[2] * 1e-3
    prods = 1 if args.form == "f32" else (kp or 3)
    peak = PEAK["fp32"] if args.form == "f32" else PEAK["bf16"]
    kname = "k_main_f32" if args.form == "f32" else "k_main_bf16"
    res = {
        "metric": "K-means (Lloyd) step points/s at D=128,K=1000; bf16-MFMA",
        "value": spec.n / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"bf16": "bf16", "fp8": "fp8e4m3", "f32": "f32"}[args.form],
        "data": "synthetic",
        "config": {"workload": spec.name, "n": spec.n, "d": spec.d, "k": spec.k, "storage": args.form,
                   "products": prods if args.form != "f32" else None, "centred": True, "kmeans_step": True},
        "phases_ms": {"stats": phases[0], "finalize": phases[1], "gemm_argmin": phases[2], "reduce": phases[3]},
        "inertia": inertia.item(), "moved_points": moved,
        "roofline": {"bound": "mfma", "achieved": useful / t_main / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": useful / t_main / peak, "traffic": None, "kernel": kname,
                     "issued_frac": useful * prods / t_main / peak,
                     "note": "achieved = 2*N*D*K useful flops / mean duration of the fused argmin kernel"},
    }
    if not args.no_check or not args.no_cpu:
        import oracle
        host_codes = wl.host_codes(X)
        labels_host = labels.cpu().numpy()
        cs_host = None if col_scale is None else col_scale.cpu().numpy()
    if not args.no_check:
        # FP64 means of all rows, then the nearest mean of sampled points in binary64
        t0 = time.perf_counter()
        count, V, _ = oracle.cluster_stats(host_codes, labels_host, spec.k, "sqeuclid", col_scale=cs_host)
        ne = count > 0
        mu = V[ne] / count[ne, None]
        ids = np.nonzero(ne)[0]
        idx = np.sort(np.random.default_rng(7).choice(spec.n, size=256, replace=False))
        codes = np.ascontiguousarray(host_codes[idx])
        if codes.dtype == np.uint16:    # bf16 bit patterns
            xs = (codes.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        elif codes.dtype == np.uint8:   # fp8 e4m3fn codes times the column scale (exact)
            xs = torch.from_numpy(codes).view(torch.float8_e4m3fn).double().numpy() * cs_host.astype(np.float64)
        else:
            xs = codes.astype(np.float64)
        d = ((xs[:, None, :] - mu[None, :, :]) ** 2).sum(axis=2)
        best = d.min(axis=1)
        got = out.cpu().numpy()[idx]
        pos = np.searchsorted(ids, got)
        ok = (pos < len(ids)) & (ids[np.minimum(pos, len(ids) - 1)] == got)
        d_got = np.where(ok, d[np.arange(len(idx)), np.minimum(pos, len(ids) - 1)], np.inf)
        res["check"] = {"sampled_points": int(len(idx)),
                        "label_equals_fp64_argmin": float((ids[d.argmin(axis=1)] == got).mean()),
                        "max_rel_excess_distance": float(((d_got - best) / np.maximum(best, 1e-30)).max()),
                        "oracle_stats_s": time.perf_counter() - t0}
        log(f"check: {res['check']}")
    if not args.no_cpu:
        n = min(args.cpu_sample, spec.n)
        t0 = time.perf_counter()
        oracle.kmeans_step(np.ascontiguousarray(host_codes[:n]), np.ascontiguousarray(labels_host[:n]), spec.k,
                           col_scale=cs_host)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": n / dt, "unit": "points/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"first {n} rows of {spec.name} "
                               f"({host_codes.dtype} storage), FP64 oracle K-means step, {dt:.1f} s"}
    print(json.dumps(res), flush=True)


def bench_mahalanobis(args, spec, X, col_scale, labels, dev):
    """Silhouette under d(x, y) = (x - y)^T L^T L (x - y) with a seeded random L = I + G / sqrt(D):
    the transform Z = X L^T on fp32 MFMA, then the fp32 squared Euclidean form on Z."""
    import numpy as np
    import torch

    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    lib = _lib.load()
    rng = np.random.default_rng(11)
    Lm = torch.from_numpy((np.eye(spec.d) + rng.standard_normal((spec.d, spec.d)) / np.sqrt(spec.d))
                          .astype(np.float32)).to(dev)
    nbytes = lib.silhouette_mahalanobis_workspace_bytes(spec.n, spec.d, spec.k, 0)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    s = torch.empty(spec.n, dtype=torch.float32, device=dev)
    S = torch.empty((), dtype=torch.float64, device=dev)
    dcode, stream, cs_ptr = sil._dtype_code(X), sil._stream(dev), sil._ptr(col_scale)

    def step():
        rc = lib.silhouette_mahalanobis(sil._ptr(X), dcode, cs_ptr, sil._ptr(Lm), sil._ptr(labels), spec.n,
                                        spec.d, spec.k, 0, sil._ptr(s), sil._ptr(S), sil._ptr(ws), ws.numel(),
                                        stream)
        if rc:
            raise _lib.SilhouetteError(rc, "mahalanobis step")

    log(f"timing the Mahalanobis form ({args.form} storage): warmup {args.warmup}, steps {args.steps}")
    ms, phases, _ = timed_steps(step, args.steps, args.warmup, torch)
    zb = (spec.n * spec.d * 4 + 255) // 256 * 256
    _lib.check(sil.status(ws[zb:]), "device status")
    useful = 2.0 * spec.n * spec.d * spec.k
    t_main = phases[2] * 1e-3
    transform_ms = ms - sum(phases)
    res = {
        "metric": "Mahalanobis Silhouette points/s at D=128,K=1000 (fixed M = L^T L; fp32 MFMA transform and form)",
        "value": spec.n / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": spec.name, "n": spec.n, "d": spec.d, "k": spec.k, "storage": args.form,
                   "metric": "mahalanobis", "L": "I + N(0,1)/sqrt(D), seed 11"},
        "phases_ms": {"transform": transform_ms, "stats": phases[0], "finalize": phases[1],
                      "gemm_epilogue": phases[2], "reduce": phases[3]},
        "S": S.item(),
        "roofline": {"bound": "mfma", "achieved": useful / t_main / 1e12, "peak": PEAK["fp32"] / 1e12,
                     "unit": "TFLOP/s", "frac": useful / t_main / PEAK["fp32"], "traffic": None,
                     "kernel": "k_main_f32",
                     "transform_TFLOPs": 2.0 * spec.n * spec.d * spec.d / (transform_ms * 1e-3) / 1e12},
    }
    print(json.dumps(res), flush=True)


def bench_backward(args, spec, X32, labels, dev):
    """S and dS/dX on fp32 embeddings (the differentiation workload): a forward call that keeps
    a_i, b_i and the neighbouring cluster, then the adjoint kernels.  The step is forward plus
    backward; the adjoint alone is timed with events on the library's stream and set against
    its HBM roofline (read X twice, write dX, read the saves and labels)."""
    import numpy as np
    import torch

    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    lib = _lib.load()
    metric = args.metric
    flags = _lib.SIL_FLAG_SAVE_FOR_GRAD
    ws = sil.new_workspace(spec.n, spec.d, spec.k, metric, torch.float32, flags, dev)
    S = torch.empty((), dtype=torch.float64, device=dev)
    gS = torch.ones((), dtype=torch.float64, device=dev)
    dX = torch.empty_like(X32)
    stream = sil._stream(dev)
    fwd = lib.silhouette_sqeuclid if metric == "sqeuclid" else lib.silhouette_cosine
    bwd = lib.silhouette_sqeuclid_backward if metric == "sqeuclid" else lib.silhouette_cosine_backward

    def forward():
        rc = fwd(sil._ptr(X32), 0, None, sil._ptr(labels), spec.n, spec.d, spec.k, 0, flags, None,
                 sil._ptr(S), sil._ptr(ws), ws.numel(), stream)
        if rc:
            raise _lib.SilhouetteError(rc, "forward")

    def backward():
        rc = bwd(sil._ptr(X32), 0, None, sil._ptr(labels), spec.n, spec.d, spec.k, flags, sil._ptr(gS),
                 sil._ptr(dX), sil._ptr(ws), ws.numel(), stream)
        if rc:
            raise _lib.SilhouetteError(rc, "backward")

    def step():
        forward()
        backward()

    log(f"timing forward + backward ({metric}): warmup {args.warmup}, steps {args.steps}")
    ms, phases, _ = timed_steps(step, args.steps, args.warmup, torch)
    _lib.check(sil.status(ws), "device status")
    # the adjoint alone, on the same saves
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nb = max(1, args.steps)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(nb):
        backward()
    ev1.record()
    torch.cuda.synchronize()
    bwd_ms = ev0.elapsed_time(ev1) / nb
    alg = spec.n * (12 * spec.d + 16)
    res = {
        "metric": f"Silhouette and dS/dX points/s at N={spec.n},D={spec.d},K={spec.k} (fp32, labels fixed)",
        "value": spec.n / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": spec.name, "n": spec.n, "d": spec.d, "k": spec.k, "metric": metric,
                   "storage": "f32", "step": "forward (saves) + backward"},
        "phases_ms": {"stats": phases[0], "finalize": phases[1], "gemm_epilogue": phases[2],
                      "reduce": phases[3], "backward": bwd_ms},
        "S": S.item(),
        "roofline": {"bound": "hbm", "achieved": alg / (bwd_ms * 1e-3) / 1e9, "peak": PEAK["hbm"] / 1e9,
                     "unit": "GB/s", "frac": alg / (bwd_ms * 1e-3) / PEAK["hbm"], "traffic": None,
                     "kernel": "kb_alpha + kb_accum(_slice) + kb_reduce + kb_gtab + kb_dx(4)",
                     "algorithmic_bytes": alg,
                     "note": "per point: X read twice, dX written (12 D bytes), saves and label (16 B)"},
        "dX_norm": float(dX.double().norm()),
    }
    if not args.no_cpu:
        import oracle
        n = min(args.cpu_sample, spec.n)
        Xs = X32[:n].cpu().numpy()
        ls = labels[:n].cpu().numpy()
        t0 = time.perf_counter()
        oracle.gradient(Xs, ls, spec.k, metric)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": n / dt, "unit": "points/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"first {n} rows of {spec.name}: FP64 oracle forward and gradient, {dt:.1f} s"}
    print(json.dumps(res), flush=True)


def bench_stream(args, spec, X, col_scale, labels, dev):
    """Out-of-core form: X and labels moved to pinned host memory (the device copy is freed), then
    every step streams them through the device twice in chunks.  The rate includes the PCIe
    transfers; it is not the device-resident rate of the default line."""
    import torch

    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    lib = _lib.load()
    metric = sil.METRIC[args.metric]
    ws_mem = sil.new_workspace(spec.n, spec.d, spec.k, args.metric, X.dtype, 0, dev)
    S_mem = torch.empty((), dtype=torch.float64, device=dev)
    fn_c = lib.silhouette_sqeuclid if args.metric == "sqeuclid" else lib.silhouette_cosine
    _lib.check(fn_c(sil._ptr(X), sil._dtype_code(X), sil._ptr(col_scale), sil._ptr(labels), spec.n, spec.d,
                    spec.k, args.products, 0, None, sil._ptr(S_mem), sil._ptr(ws_mem), ws_mem.numel(),
                    sil._stream(dev)), "in-memory reference")
    S_ref = S_mem.item()
    del ws_mem
    log("moving X and labels to pinned host memory")
    Xh = torch.empty(X.shape, dtype=X.dtype, pin_memory=True)
    Xh.copy_(X)
    lh = torch.empty(spec.n, dtype=torch.int32, pin_memory=True)
    lh.copy_(labels)
    dcode = sil._dtype_code(X)
    del X, labels
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    chunk = min(args.chunk_rows, spec.n)
    ws = torch.empty(sil.stream_workspace_bytes(spec.n, chunk, spec.d, spec.k, args.metric, Xh.dtype),
                     dtype=torch.uint8, device=dev)
    sh = torch.empty(spec.n, dtype=torch.float32, pin_memory=True)
    S = torch.empty((), dtype=torch.float64, device=dev)
    stream, cs_ptr = sil._stream(dev), sil._ptr(col_scale)

    def step():
        rc = lib.silhouette_stream(metric, ctypes.c_void_p(Xh.data_ptr()), dcode, cs_ptr,
                                   ctypes.c_void_p(lh.data_ptr()), spec.n, spec.d, spec.k, args.products, 0,
                                   ctypes.c_void_p(sh.data_ptr()), sil._ptr(S), chunk, sil._ptr(ws), ws.numel(),
                                   stream)
        if rc:
            raise _lib.SilhouetteError(rc, "stream step")

    log(f"timing the out-of-core form: chunk {chunk} rows, warmup {args.warmup}, steps {args.steps}")
    ms, _, wall = timed_steps(step, args.steps, args.warmup, torch)
    _lib.check(sil.status(ws), "device status")
    esz = Xh.element_size()
    h2d = 2 * (spec.n * spec.d * esz + 4 * spec.n)
    d2h = 4 * spec.n
    res = {
        "metric": "Out-of-core Silhouette points/s at D=128,K=1000 (X in pinned host memory, PCIe-inclusive)",
        "value": spec.n / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"bf16": "bf16", "fp8": "fp8e4m3", "f32": "f32"}[args.form],
        "data": "synthetic",
        "config": {"workload": spec.name, "n": spec.n, "d": spec.d, "k": spec.k, "metric": args.metric,
                   "storage": args.form, "products": args.products if args.form != "f32" else None,
                   "chunk_rows": chunk, "device_workspace_gb": ws.numel() / 1e9,
                   "host_bytes_gb": (Xh.numel() * esz + 4 * spec.n) / 1e9},
        "S": S.item(), "dS_vs_in_memory": abs(S.item() - S_ref),
        "transfer": {"h2d_bytes": h2d, "d2h_bytes": d2h, "h2d_GBps": h2d / (ms * 1e-3) / 1e9,
                     "note": "X and labels cross PCIe twice (statistics pass, then scoring pass)"},
    }
    print(json.dumps(res), flush=True)


def offset_ratio(X32):
    """|m| / rms |x - m| of the data (m the global mean): the folded centring's cross-term error
    scales with |x| <= |m| + |x - m| where the three-product form's scales with |x - m|."""
    import torch
    m = torch.zeros(X32.shape[1], dtype=torch.float64, device=X32.device)
    ss = torch.zeros((), dtype=torch.float64, device=X32.device)
    step = 1 << 22
    for r0 in range(0, X32.shape[0], step):
        m += X32[r0:r0 + step].double().sum(0)
    m /= X32.shape[0]
    for r0 in range(0, X32.shape[0], step):
        ss += ((X32[r0:r0 + step].double() - m) ** 2).sum()
    return float(m.norm() / torch.sqrt(ss / X32.shape[0]))


def stats_kernel(args, spec):
    """Name of the statistics pass's reduction kernel for this run: whole-wave rows for fp32 / bf16
    rows of 256, 512 or 1024 bytes and fp8 rows of 128 or 256 bytes, 16-byte chunks otherwise."""
    rb = spec.d * {"f32": 4, "bf16": 2, "fp8": 1}[args.form]
    row = rb in (256, 512, 1024) if args.form != "fp8" else spec.d in (128, 256)
    return "k_segreduce_row" if row else "k_segreduce_vec"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="blobs-50m-d128-k1000",
                    help="a named blob workload, or ksweep (the batched k-sweep, its own JSON line)")
    ap.add_argument("--metric", default="sqeuclid", choices=["sqeuclid", "cosine", "kl"])
    ap.add_argument("--form", default="bf16", choices=["bf16", "fp8", "f32"])
    ap.add_argument("--products", type=int, default=0,
                    help="bf16/fp8 split products (0: 2, where x - fp8: its codes - enters the GEMM "
                         "exact)")
    ap.add_argument("--stream", action="store_true",
                    help="out-of-core: X and labels in pinned host memory, streamed in chunks")
    ap.add_argument("--chunk-rows", type=int, default=4_000_000)
    ap.add_argument("--mahalanobis", action="store_true",
                    help="the Silhouette under a fixed Mahalanobis distance (M = L^T L, random L)")
    ap.add_argument("--backward", action="store_true",
                    help="forward + adjoint on the differentiation workload (blobs-1m-d256-k64, fp32)")
    ap.add_argument("--kmeans", action="store_true",
                    help="time one K-means (Lloyd) step on the workload instead of the Silhouette")
    ap.add_argument("--euclid-approx", action="store_true",
                    help="the approximate Euclidean form (square roots of the mean squared distances)")
    ap.add_argument("--fp32-steps", type=int, default=4)
    ap.add_argument("--x3-steps", type=int, default=10, help="steps of the BF16x3 comparison")
    ap.add_argument("--no-x3", action="store_true", help="skip the BF16x3 comparison")
    ap.add_argument("--no-fp32", action="store_true", help="skip the fp32-form comparison")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle check")
    ap.add_argument("--check", default="full", choices=["full", "sampled"],
                    help="full: every s_i and S against the whole FP64 oracle (about 2 minutes of "
                         "host time at the default workload); sampled: 256 points")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-screen", action="store_true",
                    help="squared Euclidean, bf16, two products: the plain two-product sweep for every row")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the measured copy / GEMM peaks and the small workload's latency")
    ap.add_argument("--cpu-sample", type=int, default=4_000_000)
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a plain 2 GiB device copy (reference for the traffic counters)")
    ap.add_argument("--n", type=int, default=0, help="override N (testing only)")
    ap.add_argument("--k", type=int, default=0, help="override K (testing only)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_steps(fn, steps, warmup, torch):
    """Run `warmup` untimed calls, then `steps` timed ones between synchronisations; returns
    (ms per step, phase ms per step [4])."""
    from paper_2303_14102_amd import _lib
    lib = _lib.load()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    _lib.check(lib.silhouette_profile_begin(steps), "profile_begin")
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    ms = (ctypes.c_float * 4)()
    n = ctypes.c_int32()
    _lib.check(lib.silhouette_profile_end(ms, ctypes.byref(n)), "profile_end")
    total = start.elapsed_time(stop)
    return total / steps, [v / max(1, n.value) for v in ms], wall / steps


def measured_peaks(torch, dev):
    """What this GPU reaches on plain library work, beside the datasheet peaks: a 2 GiB
    device-to-device copy (bytes read + written per second) and a bf16 8192^3 matrix product
    (hipBLASLt through torch.matmul).  Measurement references only; the Silhouette path uses
    neither."""
    src = torch.empty(1 << 31, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    a = torch.randn(8192, 8192, device=dev).to(torch.bfloat16)
    b = torch.randn(8192, 8192, device=dev).to(torch.bfloat16)

    def best_ms(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    t_copy = best_ms(lambda: dst.copy_(src))
    t_mm = best_ms(lambda: torch.matmul(a, b))
    out = {"hbm_copy_GBps": 2 * src.numel() / (t_copy * 1e-3) / 1e9,
           "bf16_gemm_TFLOPs": 2 * 8192 ** 3 / (t_mm * 1e-3) / 1e12,
           "how": "best of 10: 2 GiB device copy (read + write bytes); bf16 8192^3 torch.matmul"}
    del src, dst, a, b
    torch.cuda.empty_cache()
    return out


def latency_c1(torch, dev):
    """The small plain-method workload (N = 10,000, D = 8, K = 4, fp32): microseconds per call,
    launched eagerly through the C ABI, and replayed from a captured graph of the same call."""
    from paper_2303_14102_amd import binding as sil
    from paper_2303_14102_amd import workloads as wl
    spec = wl.WORKLOADS["blobs-10k-d8-k4"]
    b = wl.make_blobs(spec, dev)
    res = {"workload": spec.name}
    for metric in ("sqeuclid", "cosine"):
        ws = sil.new_workspace(spec.n, spec.d, spec.k, metric, torch.float32, 0, dev)
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            for _ in range(20):
                sil.silhouette(b.X, b.labels, spec.k, metric, workspace=ws)
            n = 200
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            side.synchronize()
            t0 = time.perf_counter()
            e0.record()
            for _ in range(n):
                sil.silhouette(b.X, b.labels, spec.k, metric, workspace=ws)
            e1.record()
            side.synchronize()
            eager_wall = (time.perf_counter() - t0) / n * 1e6
            eager = e0.elapsed_time(e1) / n * 1e3
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                sil.silhouette(b.X, b.labels, spec.k, metric, workspace=ws)
            for _ in range(20):
                g.replay()
            side.synchronize()
            e0.record()
            for _ in range(n):
                g.replay()
            e1.record()
            side.synchronize()
            graph = e0.elapsed_time(e1) / n * 1e3
        torch.cuda.current_stream(dev).wait_stream(side)
        res[metric] = {"eager_us_per_call": eager, "eager_wall_us_per_call": eager_wall,
                       "graph_replay_us_per_call": graph, "points_per_s_graph": spec.n / (graph * 1e-6)}
        del g, ws
    return res


def cpu_baseline(spec, X_host_codes, labels_host, metric, col_scale, n_sample):
    import numpy as np
    import oracle
    n = min(n_sample, len(labels_host))
    Xs = np.ascontiguousarray(X_host_codes[:n])
    ls = np.ascontiguousarray(labels_host[:n])
    t0 = time.perf_counter()
    oracle.silhouette(Xs, ls, spec.k, metric, col_scale=col_scale)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"first {n} rows of {spec.name} ({X_host_codes.dtype} storage), whole FP64 "
                      f"oracle (statistics pass + every point), {dt:.1f} s"}


def bench_ksweep(args):
    """The batched k-sweep: 32 data sets x 8 labelings in one tuned plan, timed as hipGraph replays."""
    import numpy as np
    import torch

    from paper_2303_14102_amd import BatchedSilhouette
    from paper_2303_14102_amd import workloads as wl

    dev = torch.device("cuda:0")
    log("generating the k-sweep workload (32 data sets x 8 labelings)")
    t0 = time.perf_counter()
    data = wl.make_ksweep(device=dev)
    probs = [(ds.X, lab, k, args.metric) for ds in data for k, lab in ds.labelings]
    torch.cuda.synchronize()
    n_points = sum(p[0].shape[0] for p in probs)
    log(f"{len(probs)} problems, {n_points} points, generated in {time.perf_counter() - t0:.1f} s")
    batch = BatchedSilhouette(probs)
    t_main = batch.tune()
    cfg = batch.config()
    log(f"tuned: persistent launch {t_main:.3f} ms, {cfg}")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    batch.capture(side)
    for _ in range(args.warmup):
        batch.replay(side)
    side.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(side)
    for _ in range(args.steps):
        batch.replay(side)
    e1.record(side)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    st = batch.status()
    if any(st):
        raise RuntimeError(f"device status {st}")
    # roofline of the persistent kernel: useful flops, and the per-problem roofline time summed
    flops = sum(2.0 * p[0].shape[0] * p[0].shape[1] * p[2] for p in probs)
    roof_t = sum(max(2.0 * p[0].shape[0] * p[0].shape[1] * p[2] / PEAK["fp32"],
                     (p[0].shape[0] * (4 * p[0].shape[1] + 12)) / PEAK["hbm"]) for p in probs)
    out = {
        "metric": "Silhouette points/s, batched k-sweep (256 labelings, one persistent launch)",
        "value": n_points / (ms * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ksweep-32x8", "problems": len(probs), "points": n_points,
                   "metric": args.metric, "tuned": cfg, "replay": "hipGraph"},
        "roofline": {"bound": "mfma", "achieved": flops / (t_main * 1e-3) / 1e12, "peak": PEAK["fp32"] / 1e12,
                     "unit": "TFLOP/s", "frac": flops / (t_main * 1e-3) / PEAK["fp32"], "traffic": None,
                     "kernel": "k_main_f32_batched", "kernel_ms": t_main,
                     "summed_problem_roofline_ms": roof_t * 1e3,
                     "frac_of_summed_roofline": roof_t * 1e3 / t_main},
    }
    if not args.no_cpu:
        import oracle
        # the oracle on whole problems, in batch order, until about 15 s of CPU time
        t0 = time.perf_counter()
        done = 0
        used = 0
        for X, lab, k, metric in probs:
            if time.perf_counter() - t0 > 15.0:
                break
            oracle.silhouette(X.cpu().numpy(), lab.cpu().numpy(), k, metric)
            done += X.shape[0]
            used += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done / dt, "unit": "points/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"the first {used} problems of the batch ({done} points), whole FP64 "
                                         f"oracle each, {dt:.1f} s (includes the host copies)"}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.products == 0:
        args.products = 2
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU form is a design note, not a measured path)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2303_14102_amd import binding as sil
    from paper_2303_14102_amd import workloads as wl

    if args.workload == "ksweep":
        return bench_ksweep(args)
    dev = torch.device("cuda:0")
    if args.backward:
        if args.workload == "blobs-50m-d128-k1000":
            args.workload = "blobs-1m-d256-k64"
        args.form = "f32"
        if args.metric not in ("sqeuclid", "cosine"):
            sys.exit("--backward: squared Euclidean or cosine")
    spec = wl.WORKLOADS[args.workload]
    if args.n:
        spec = wl.scaled(spec, args.n)
    if args.k:
        import dataclasses
        spec = dataclasses.replace(spec, k=args.k, name=f"{spec.name}@k{args.k}")
    log(f"generating {spec.name} N={spec.n} D={spec.d} K={spec.k}")
    t0 = time.perf_counter()
    blobs = wl.make_blobs(spec, dev)
    X32, labels = blobs.X, blobs.labels
    if args.metric == "kl":
        # the generalized KL divergence needs positive vectors: exponentiated blob coordinates
        if args.form == "fp8" or args.kmeans or args.mahalanobis or args.stream:
            sys.exit("--metric kl runs the plain Silhouette with fp32 or bf16 storage")
        X32 = torch.exp(X32 * 0.25)
    col_scale = None
    if args.form == "bf16":
        X = wl.to_bf16(X32)
    elif args.form == "fp8":
        X, col_scale = wl.to_fp8_e4m3(X32)
    else:
        X = X32
    torch.cuda.synchronize()
    log(f"generated in {time.perf_counter() - t0:.1f} s")

    if args.backward:
        return bench_backward(args, spec, X32, labels, dev)
    if args.kmeans:
        return bench_kmeans(args, spec, X, col_scale, labels, dev)
    if args.mahalanobis:
        return bench_mahalanobis(args, spec, X, col_scale, labels, dev)
    if args.stream:
        del X32, blobs
        return bench_stream(args, spec, X, col_scale, labels, dev)

    ws = sil.new_workspace(spec.n, spec.d, spec.k, args.metric, X.dtype, 0, dev)
    s = torch.empty(spec.n, dtype=torch.float32, device=dev)
    S = torch.empty((), dtype=torch.float64, device=dev)

    from paper_2303_14102_amd import _lib
    lib = _lib.load()
    fn_c = {"sqeuclid": lib.silhouette_sqeuclid, "cosine": lib.silhouette_cosine,
            "kl": lib.silhouette_kl}[args.metric]
    if args.euclid_approx and args.metric != "sqeuclid":
        sys.exit("--euclid-approx applies to the squared Euclidean entry point")
    flags = (_lib.SIL_FLAG_EUCLID_APPROX if args.euclid_approx else 0) | (
        _lib.SIL_FLAG_NO_SCREEN if args.no_screen else 0)
    ref_metric = "euclid_approx" if args.euclid_approx else args.metric
    dcode = sil._dtype_code(X)
    stream = sil._stream(dev)
    cs_ptr = sil._ptr(col_scale)

    def step():
        rc = fn_c(sil._ptr(X), dcode, cs_ptr, sil._ptr(labels), spec.n, spec.d, spec.k, args.products, flags,
                  sil._ptr(s), sil._ptr(S), sil._ptr(ws), ws.numel(), stream)
        if rc:
            raise _lib.SilhouetteError(rc, "step")

    log(f"timing {args.form} form: warmup {args.warmup}, steps {args.steps}")
    ms, phases, wall = timed_steps(step, args.steps, args.warmup, torch)
    st = sil.status(ws)
    _lib.check(st, "device status")
    S_form = S.item()
    log(f"{args.form}: {ms:.3f} ms/step (wall {wall:.3f}), phases {['%.3f' % p for p in phases]}, S={S_form:.10f}")

    out = {
        "metric": ("Approximate-Euclidean " if args.euclid_approx else "")
        + ("Generalized-KL " if args.metric == "kl" else "")
        + (f"Silhouette points/s at D={spec.d},K={spec.k}; "
           + ("bf16-MFMA vs fp32 form at |dS|<1e-4" if args.form != "f32" else "fp32 form")),
        "value": spec.n / (ms * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16", "fp8": "fp8e4m3", "f32": "f32"}[args.form],
        "data": "synthetic",
        "config": {"workload": spec.name, "n": spec.n, "d": spec.d, "k": spec.k,
                   "metric": args.metric, "storage": args.form,
                   "products": args.products if args.form != "f32" else None,
                   "centred": args.metric == "sqeuclid",
                   **({"centring": "folded into c_k (x enters the GEMM exact)",
                       "mean_offset_ratio": offset_ratio(X32)}
                      if args.metric == "sqeuclid" and args.form in ("bf16", "fp8") and args.products == 2 else {}),
                   **({"normalisation": "1/|x| applied after the minimum (x enters the GEMM exact)"}
                      if args.metric == "cosine" and args.form in ("bf16", "fp8") and args.products == 2 else {}),
                   **({"euclid_approx": True} if args.euclid_approx else {}),
                   **({"data_transform": "exp(x/4) of the blob coordinates"} if args.metric == "kl" else {})},
        "phases_ms": {"stats": phases[0], "finalize": phases[1], "gemm_epilogue": phases[2],
                      "reduce": phases[3]},
        "S": S_form,
    }

    # roofline of the dominant kernel: the fused GEMM + epilogue
    useful = 2.0 * spec.n * spec.d * spec.k
    t_main = phases[2] * 1e-3
    peak = PEAK["fp32"] if args.form == "f32" else PEAK["bf16"]
    prods = 1 if args.form == "f32" else args.products
    kname = "k_main_bf16" if args.form != "f32" else "k_main_f32"
    screened = (args.form in ("bf16", "fp8") and args.metric == "sqeuclid" and args.products == 2
                and spec.d <= 128 and (args.form == "bf16" or spec.d % 8 == 0) and not args.no_screen)
    issued = useful * prods
    variant = f"{args.form}/{args.metric}/p{args.products}" + ("/noscreen" if args.no_screen else "")
    note = ("achieved = 2*N*D*K useful flops / mean duration of the fused kernel; "
            "issued_frac counts every split product")
    if screened:
        fb = sil.fallback_rows(ws)
        # the screen: one fp16 product over D coordinates for every row (the constant is the
        # accumulators' initial value); the two-product kernel over the listed rows
        depth = -(-spec.d // 16) * 16
        issued = 2.0 * spec.n * spec.k * depth + 2.0 * 2.0 * fb * spec.k * depth
        kname = "k_main_screen"
        note = ("achieved = 2*N*D*K useful flops / mean duration of the fused phase (the fp16 screen "
                "kernel, then the two-product kernel over the rows it leaves); issued_frac counts the "
                "screen's padded depth and the fallback's two products")
        out["screen"] = {"fallback_rows": fb, "fallback_frac": fb / spec.n,
                         "kernels": ["k_main_screen", "k_main_fallback", "k_fb_sum"]}
    out["roofline"] = {"bound": "mfma", "achieved": useful / t_main / 1e12, "peak": peak / 1e12,
                       "unit": "TFLOP/s", "frac": useful / t_main / peak,
                       "traffic": measured_traffic(kname, spec.name, variant),
                       "kernel": kname,
                       "issued_frac": issued / t_main / peak,
                       "note": note}
    stats_bytes = spec.n * spec.d * X.element_size() + 4 * spec.n
    out["stats_pass"] = {"bound": "hbm", "algorithmic_bytes": stats_bytes,
                         "achieved_GBps": stats_bytes / (phases[0] * 1e-3) / 1e9,
                         "frac": stats_bytes / (phases[0] * 1e-3) / PEAK["hbm"],
                         "traffic": measured_traffic(stats_kernel(args, spec), spec.name, variant)}

    if args.calibrate:
        # a plain device copy of known size: the reference for the FETCH_SIZE / WRITE_SIZE counters
        src = torch.empty(2 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the BF16x3 form (three products on the centred / normalised point) in the same run: the
    # two-product form on the exact x is the default only at the same accuracy
    s3 = None
    if args.form in ("bf16", "fp8") and args.products == 2 and args.metric in ("sqeuclid", "cosine") \
            and not args.no_x3:
        s3 = torch.empty(spec.n, dtype=torch.float32, device=dev)
        S3 = torch.empty((), dtype=torch.float64, device=dev)

        def step3():
            rc = fn_c(sil._ptr(X), dcode, cs_ptr, sil._ptr(labels), spec.n, spec.d, spec.k, 3, flags,
                      sil._ptr(s3), sil._ptr(S3), sil._ptr(ws), ws.numel(), stream)
            if rc:
                raise _lib.SilhouetteError(rc, "step3")

        log(f"timing the BF16x3 form: {args.x3_steps} steps")
        ms3, ph3, _ = timed_steps(step3, args.x3_steps, 1, torch)
        _lib.check(sil.status(ws), "device status BF16x3")
        out["bf16x3_form"] = {"products": 3, "ms_per_step": ms3, "value": spec.n / (ms3 * 1e-3),
                              "S": S3.item(), "gemm_epilogue_ms": ph3[2],
                              "frac": useful / (ph3[2] * 1e-3) / peak,
                              "dS_vs_two_product_form": abs(S3.item() - S_form)}
        log(f"BF16x3 form: {ms3:.3f} ms/step, S={S3.item():.10f}")

    if not args.no_fp32 and args.form != "f32":
        ws32 = sil.new_workspace(spec.n, spec.d, spec.k, args.metric, torch.float32, 0, dev)
        S32 = torch.empty((), dtype=torch.float64, device=dev)

        def step32():
            rc = fn_c(sil._ptr(X32), 0, None, sil._ptr(labels), spec.n, spec.d, spec.k, 0, flags,
                      None, sil._ptr(S32), sil._ptr(ws32), ws32.numel(), stream)
            if rc:
                raise _lib.SilhouetteError(rc, "step32")

        log(f"timing fp32 form: {args.fp32_steps} steps")
        ms32, ph32, _ = timed_steps(step32, args.fp32_steps, 1, torch)
        _lib.check(sil.status(ws32), "device status fp32")
        out["fp32_form"] = {"ms_per_step": ms32, "value": spec.n / (ms32 * 1e-3), "S": S32.item(),
                            "gemm_epilogue_ms": ph32[2],
                            "gemm_frac_of_fp32_peak": useful / (ph32[2] * 1e-3) / PEAK["fp32"]}
        out["speedup_vs_fp32_form"] = ms32 / ms
        out["dS_vs_fp32_form"] = abs(S_form - S32.item())
        if s3 is not None:
            out["bf16x3_form"]["dS_vs_fp32_form"] = abs(out["bf16x3_form"]["S"] - S32.item())
        log(f"fp32 form: {ms32:.3f} ms/step, S={S32.item():.10f}")
        del ws32

    if not args.no_extras:
        # what this machine reaches on plain library work, and the small workload's call latency
        log("measured peaks: device copy and a bf16 library GEMM")
        mp = measured_peaks(torch, dev)
        out["measured_peaks"] = mp
        if args.form != "f32":
            out["roofline"]["frac_vs_measured_gemm"] = out["roofline"]["achieved"] * 1e12 / (
                mp["bf16_gemm_TFLOPs"] * 1e12)
        out["stats_pass"]["frac_vs_measured_copy"] = out["stats_pass"]["achieved_GBps"] / mp["hbm_copy_GBps"]
        log(f"measured peaks: {mp}")
        log("latency of the small workload: eager and graph-replayed calls")
        out["latency_small"] = latency_c1(torch, dev)
        log(f"latency: {out['latency_small']}")

    host_codes = None
    if not args.no_check or not args.no_cpu:
        host_codes = wl.host_codes(X)
        labels_host = labels.cpu().numpy()
        cs_host = None if col_scale is None else col_scale.cpu().numpy()

    if not args.no_check and args.check == "full":
        import oracle
        log(f"oracle check: the whole FP64 oracle over all {spec.n} rows")
        t0 = time.perf_counter()
        # the oracle's two passes (orc_silhouette's arithmetic), the second a chunk of rows at a
        # time so that progress shows; S is the index-order sum of s_i over N, as it forms it
        stats = oracle.cluster_stats(host_codes, labels_host, spec.k, ref_metric, col_scale=cs_host)
        s_ref = np.empty(spec.n)
        for i0 in range(0, spec.n, 5_000_000):
            idx = np.arange(i0, min(spec.n, i0 + 5_000_000), dtype=np.int64)
            s_ref[idx] = oracle.scores_at(host_codes, labels_host, spec.k, idx, stats, ref_metric,
                                          col_scale=cs_host)[0]
            log(f"oracle rows [{i0}, {idx[-1] + 1}): {time.perf_counter() - t0:.1f} s")
        S_ref = float(np.cumsum(s_ref)[-1]) / spec.n
        t_orc = time.perf_counter() - t0
        s_all = s.cpu().numpy().astype(np.float64)
        out["check"] = {"points": int(spec.n), "oracle": "whole FP64 oracle on the same stored input",
                        "S_oracle": S_ref, "dS_vs_oracle": abs(S_form - S_ref),
                        "max_abs_ds": float(np.abs(s_all - s_ref).max()),
                        "S_vs_sum_of_s": abs(S_form - s_all.sum() / spec.n),
                        "oracle_s": t_orc}
        del s_all
        if s3 is not None:
            s3_all = s3.cpu().numpy().astype(np.float64)
            out["bf16x3_form"]["dS_vs_oracle"] = abs(out["bf16x3_form"]["S"] - S_ref)
            out["bf16x3_form"]["max_abs_ds"] = float(np.abs(s3_all - s_ref).max())
            del s3_all
        del s_ref
        log(f"check: {out['check']}")
    elif not args.no_check:
        import oracle
        log("oracle check on sampled points (FP64 statistics over the full data)")
        t0 = time.perf_counter()
        stats = oracle.cluster_stats(host_codes, labels_host, spec.k, ref_metric, col_scale=cs_host)
        idx = np.random.default_rng(7).choice(spec.n, size=256, replace=False)
        s_ref, a_ref, b_ref, _ = oracle.scores_at(host_codes, labels_host, spec.k, idx, stats,
                                                  ref_metric, col_scale=cs_host)
        s_gpu = s.cpu().numpy()[idx].astype(np.float64)
        s_all = s.cpu().numpy().astype(np.float64)
        out["check"] = {"sampled_points": int(len(idx)),
                        "max_abs_ds_sampled": float(np.abs(s_gpu - s_ref).max()),
                        "S_vs_sum_of_s": abs(S_form - s_all.sum() / spec.n),
                        "oracle_stats_s": time.perf_counter() - t0}
        if s3 is not None:
            out["bf16x3_form"]["max_abs_ds_sampled"] = float(
                np.abs(s3.cpu().numpy()[idx].astype(np.float64) - s_ref).max())
        log(f"check: {out['check']}")

    if not args.no_cpu:
        log(f"cpu baseline: oracle on {args.cpu_sample} rows")
        out["cpu_baseline"] = cpu_baseline(spec, host_codes, labels_host, ref_metric, cs_host, args.cpu_sample)
        log(f"cpu baseline: {out['cpu_baseline']}")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
