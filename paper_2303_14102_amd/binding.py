"""Torch-facing wrappers of the C ABI (include/silhouette.h).

torch supplies device memory and the current HIP stream; the library does all the work.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

from . import _lib as L

METRIC = {"sqeuclid": L.SIL_SQEUCLID, "cosine": L.SIL_COSINE, "kl": L.SIL_KL}


def _dtype_code(X: torch.Tensor) -> int:
    if X.dtype == torch.float32:
        return L.SIL_F32
    if X.dtype == torch.bfloat16:
        return L.SIL_BF16
    if X.dtype == torch.float8_e4m3fn:
        return L.SIL_FP8_E4M3
    raise TypeError(f"unsupported X dtype {X.dtype} (float32, bfloat16 or float8_e4m3fn)")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_inputs(X, labels, col_scale):
    if X.device.type != "cuda" or labels.device != X.device:
        raise ValueError("X and labels must be on the same GPU")
    if X.dim() != 2 or not X.is_contiguous():
        raise ValueError("X must be a contiguous [N, D] tensor")
    if X.data_ptr() % 16:
        raise ValueError("X must start at a 16-byte aligned address (a fresh tensor or X.clone())")
    if labels.dtype != torch.int32 or labels.shape != (X.shape[0],) or not labels.is_contiguous():
        raise ValueError("labels must be a contiguous int32 [N] tensor")
    if X.dtype == torch.float8_e4m3fn:
        _check_col_scale(col_scale, X.shape[1], X.device)


def _check_col_scale(col_scale, D, device):
    """fp8 storage: the kernels read col_scale as D consecutive float32 values in device memory,
    so anything else (a host tensor, a strided view, another dtype or length) is refused here,
    before any launch."""
    if (col_scale is None or col_scale.dtype != torch.float32 or tuple(col_scale.shape) != (D,)
            or not col_scale.is_contiguous() or col_scale.device != device):
        raise ValueError("fp8 X needs a contiguous float32 [D] col_scale on the same device as X")


def workspace_bytes(N: int, D: int, K: int, metric: str = "sqeuclid", dtype=torch.float32,
                    flags: int = 0) -> int:
    code = {torch.float32: L.SIL_F32, torch.bfloat16: L.SIL_BF16,
            torch.float8_e4m3fn: L.SIL_FP8_E4M3}[dtype]
    n = L.load().silhouette_workspace_bytes(N, D, K, METRIC[metric], code, flags)
    if n == 0:
        raise ValueError(f"shape out of range: N={N} D={D} K={K}")
    return n


def new_workspace(N: int, D: int, K: int, metric: str, dtype, flags: int, device) -> torch.Tensor:
    nbytes = workspace_bytes(N, D, K, metric, dtype, flags)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def silhouette(X: torch.Tensor, labels: torch.Tensor, K: int, metric: str = "sqeuclid", *,
               products: int = 0, centre: bool = True, col_scale: Optional[torch.Tensor] = None,
               want_s: bool = True, save_for_grad: bool = False, euclid_approx: bool = False,
               screen: bool = True, workspace: Optional[torch.Tensor] = None,
               check_status: bool = False):
    """Per-point s_i (float32 [N] or None) and the mean S (float64 0-d tensor on the device).

    metric: "sqeuclid", "cosine" or "kl" (the generalized Kullback-Leibler divergence of positive
    vectors, fp32 or bf16 storage).  products: bf16/fp8 cross-term products (1, 2, 3; 0 = library
    default).  centre: subtract the global mean first (squared Euclidean only).  euclid_approx:
    the approximate Euclidean form (square roots of the point-to-cluster mean squared distances;
    squared Euclidean only).  screen: the one-product screen of the squared Euclidean bf16
    two-product form (False: the plain two-product sweep for every point).
    workspace: a uint8 device tensor of at least workspace_bytes(...) bytes, reused across
    calls; allocated here when None.
    """
    _check_inputs(X, labels, col_scale)
    N, D = X.shape
    flags = ((0 if centre else L.SIL_FLAG_NO_CENTRE) | (L.SIL_FLAG_SAVE_FOR_GRAD if save_for_grad else 0)
             | (L.SIL_FLAG_EUCLID_APPROX if euclid_approx else 0) | (0 if screen else L.SIL_FLAG_NO_SCREEN))
    if workspace is None:
        workspace = new_workspace(N, D, K, metric, X.dtype, flags, X.device)
    s = torch.empty(N, dtype=torch.float32, device=X.device) if want_s else None
    S = torch.empty((), dtype=torch.float64, device=X.device)
    lib = L.load()
    fn = {"sqeuclid": lib.silhouette_sqeuclid, "cosine": lib.silhouette_cosine, "kl": lib.silhouette_kl}[metric]
    rc = fn(_ptr(X), _dtype_code(X), _ptr(col_scale), _ptr(labels), N, D, int(K), int(products), flags,
            _ptr(s), _ptr(S), _ptr(workspace), workspace.numel(), _stream(X.device))
    L.check(rc, f"silhouette_{metric}")
    if check_status:
        L.check(status(workspace), f"silhouette_{metric} (device)")
    return s, S


def sqeuclid_noalloc(X: torch.Tensor, labels: torch.Tensor, K: int, *, products: int = 0,
                     centre: bool = True, col_scale: Optional[torch.Tensor] = None,
                     s: Optional[torch.Tensor] = None, S: Optional[torch.Tensor] = None,
                     status: Optional[torch.Tensor] = None):
    """silhouette_sqeuclid_noalloc: the squared Euclidean Silhouette with the library's static
    per-GPU scratch as the workspace.  s (float32 [N] or None), S (float64 0-d) and status (int32
    [1] or None) are written in place when given (allocated here otherwise), so that a caller that
    must not allocate passes all three."""
    _check_inputs(X, labels, col_scale)
    N, D = X.shape
    if S is None:
        S = torch.empty((), dtype=torch.float64, device=X.device)
    for t, dt, shape in ((s, torch.float32, (N,)), (S, torch.float64, ()), (status, torch.int32, (1,))):
        if t is not None and (t.dtype != dt or tuple(t.shape) != shape or t.device != X.device
                              or not t.is_contiguous()):
            raise ValueError(f"output must be a contiguous {dt} tensor of shape {shape} on X's device")
    flags = 0 if centre else L.SIL_FLAG_NO_CENTRE
    rc = L.load().silhouette_sqeuclid_noalloc(_ptr(X), _dtype_code(X), _ptr(col_scale), _ptr(labels), N, D,
                                              int(K), int(products), flags, _ptr(s), _ptr(S), _ptr(status),
                                              _stream(X.device))
    L.check(rc, "silhouette_sqeuclid_noalloc")
    return s, S, status


def cluster_stats(X: torch.Tensor, labels: torch.Tensor, K: int, metric: str = "sqeuclid", *,
                  col_scale: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None):
    """(count int32 [K], V float64 [K, D], psi float64 [K]) from one pass over X."""
    _check_inputs(X, labels, col_scale)
    N, D = X.shape
    if workspace is None:
        workspace = new_workspace(N, D, K, metric, X.dtype, 0, X.device)
    count = torch.empty(K, dtype=torch.int32, device=X.device)
    V = torch.empty((K, D), dtype=torch.float64, device=X.device)
    psi = torch.empty(K, dtype=torch.float64, device=X.device)
    rc = L.load().silhouette_cluster_stats(_ptr(X), _dtype_code(X), _ptr(col_scale), _ptr(labels), N, D,
                                           int(K), METRIC[metric], _ptr(count), _ptr(V), _ptr(psi),
                                           _ptr(workspace), workspace.numel(), _stream(X.device))
    L.check(rc, "silhouette_cluster_stats")
    return count, V, psi


def kmeans_step(X: torch.Tensor, labels: torch.Tensor, K: int, *, products: int = 0,
                centre: bool = True, col_scale: Optional[torch.Tensor] = None,
                labels_out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                check_status: bool = False):
    """One K-means (Lloyd) step: (new labels int32 [N], inertia float64 0-d tensor), both on the
    device.  labels_out may be `labels` itself (an in-place step)."""
    _check_inputs(X, labels, col_scale)
    N, D = X.shape
    flags = 0 if centre else L.SIL_FLAG_NO_CENTRE
    if workspace is None:
        workspace = new_workspace(N, D, K, "sqeuclid", X.dtype, flags, X.device)
    if labels_out is None:
        labels_out = torch.empty(N, dtype=torch.int32, device=X.device)
    inertia = torch.empty((), dtype=torch.float64, device=X.device)
    rc = L.load().silhouette_kmeans_step(_ptr(X), _dtype_code(X), _ptr(col_scale), _ptr(labels), N, D,
                                         int(K), int(products), flags, _ptr(labels_out), _ptr(inertia),
                                         _ptr(workspace), workspace.numel(), _stream(X.device))
    L.check(rc, "silhouette_kmeans_step")
    if check_status:
        L.check(status(workspace), "silhouette_kmeans_step (device)")
    return labels_out, inertia


def silhouette_mahalanobis(X: torch.Tensor, labels: torch.Tensor, K: int, L_mat: torch.Tensor, *,
                           centre: bool = True, col_scale: Optional[torch.Tensor] = None, want_s: bool = True,
                           workspace: Optional[torch.Tensor] = None, check_status: bool = False):
    """Silhouette under d(x, y) = (x - y)^T M (x - y) with M = L_mat^T L_mat (L_mat float32 [D, D] on the
    device): (s float32 [N] or None, S float64 0-d tensor)."""
    _check_inputs(X, labels, col_scale)
    N, D = X.shape
    if L_mat.dtype != torch.float32 or L_mat.shape != (D, D) or L_mat.device != X.device:
        raise ValueError("L_mat must be a float32 [D, D] tensor on the device of X")
    L_mat = L_mat.contiguous()
    flags = 0 if centre else L.SIL_FLAG_NO_CENTRE
    if workspace is None:
        nbytes = L.load().silhouette_mahalanobis_workspace_bytes(N, D, int(K), flags)
        if nbytes == 0:
            raise ValueError(f"shape out of range: N={N} D={D} K={K}")
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
    s = torch.empty(N, dtype=torch.float32, device=X.device) if want_s else None
    S = torch.empty((), dtype=torch.float64, device=X.device)
    rc = L.load().silhouette_mahalanobis(_ptr(X), _dtype_code(X), _ptr(col_scale), _ptr(L_mat), _ptr(labels),
                                         N, D, int(K), flags, _ptr(s), _ptr(S), _ptr(workspace),
                                         workspace.numel(), _stream(X.device))
    L.check(rc, "silhouette_mahalanobis")
    if check_status:
        zb = (N * D * 4 + 255) // 256 * 256
        L.check(status(workspace[zb:]), "silhouette_mahalanobis (device)")
    return s, S


def stream_workspace_bytes(N: int, chunk_rows: int, D: int, K: int, metric: str = "sqeuclid",
                           dtype=torch.float32, flags: int = 0) -> int:
    code = {torch.float32: L.SIL_F32, torch.bfloat16: L.SIL_BF16,
            torch.float8_e4m3fn: L.SIL_FP8_E4M3}[dtype]
    n = L.load().silhouette_stream_workspace_bytes(N, chunk_rows, D, K, METRIC[metric], code, flags)
    if n == 0:
        raise ValueError(f"shape out of range: N={N} chunk_rows={chunk_rows} D={D} K={K}")
    return n


def silhouette_stream(X_host: torch.Tensor, labels_host: torch.Tensor, K: int, metric: str = "sqeuclid", *,
                      chunk_rows: int, products: int = 0, centre: bool = True,
                      col_scale: Optional[torch.Tensor] = None, want_s: bool = True,
                      euclid_approx: bool = False, workspace: Optional[torch.Tensor] = None,
                      device: Optional[torch.device] = None, sync: bool = True, check_status: bool = False):
    """Out-of-core evaluation: X_host [N, D] and labels_host int32 [N] stay in host memory (pinned for
    the uploads to overlap the kernels) and are streamed in chunks of `chunk_rows` rows.  Returns
    (s float32 [N] in pinned host memory or None, S float64 0-d tensor on the device).  With
    sync=False the call returns after enqueueing: the host tensors must then be kept alive and
    unchanged until the current stream completes."""
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    if device.type == "cuda" and device.index is None:
        device = torch.device("cuda", torch.cuda.current_device())
    if X_host.device.type != "cpu" or labels_host.device.type != "cpu":
        raise ValueError("X_host and labels_host must be host tensors")
    if X_host.dim() != 2 or not X_host.is_contiguous():
        raise ValueError("X_host must be a contiguous [N, D] tensor")
    if labels_host.dtype != torch.int32 or labels_host.shape != (X_host.shape[0],) or not labels_host.is_contiguous():
        raise ValueError("labels_host must be a contiguous int32 [N] tensor")
    if X_host.dtype == torch.float8_e4m3fn:
        _check_col_scale(col_scale, X_host.shape[1], device)
    N, D = X_host.shape
    flags = ((0 if centre else L.SIL_FLAG_NO_CENTRE) | (L.SIL_FLAG_EUCLID_APPROX if euclid_approx else 0))
    if workspace is None:
        nbytes = stream_workspace_bytes(N, chunk_rows, D, K, metric, X_host.dtype, flags)
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
    s = torch.empty(N, dtype=torch.float32, pin_memory=True) if want_s else None
    S = torch.empty((), dtype=torch.float64, device=device)
    rc = L.load().silhouette_stream(METRIC[metric], ctypes.c_void_p(X_host.data_ptr()), _dtype_code(X_host),
                                    _ptr(col_scale), ctypes.c_void_p(labels_host.data_ptr()), N, D, int(K),
                                    int(products), flags, _ptr(s), _ptr(S), int(chunk_rows), _ptr(workspace),
                                    workspace.numel(), _stream(device))
    L.check(rc, "silhouette_stream")
    if sync:
        torch.cuda.current_stream(device).synchronize()
    if check_status:
        L.check(status(workspace), "silhouette_stream (device)")
    return s, S


def fallback_rows(workspace: torch.Tensor) -> int:
    """Rows the one-product screen of the last call on `workspace` left to the two-product
    kernel (header word 40; 0 for calls without the screen).  Synchronises the device."""
    return int(workspace[160:164].view(torch.int32).item())


def status(workspace: torch.Tensor) -> int:
    """First device-detected error of the last call on this workspace (waits for the stream)."""
    return L.load().silhouette_status(_ptr(workspace), _stream(workspace.device))


def silhouette_backward(X: torch.Tensor, labels: torch.Tensor, K: int, metric: str,
                        grad_S: torch.Tensor, workspace: torch.Tensor, *, centre: bool = True):
    """gS * dS/dX (float32 [N, D]) from the workspace of a forward call made with
    save_for_grad=True on the same inputs.  X must be float32."""
    _check_inputs(X, labels, None)
    if X.dtype != torch.float32:
        raise TypeError("the backward needs X stored float32")
    N, D = X.shape
    flags = (0 if centre else L.SIL_FLAG_NO_CENTRE) | L.SIL_FLAG_SAVE_FOR_GRAD
    gS = grad_S.to(device=X.device, dtype=torch.float64).reshape(()).contiguous()
    dX = torch.empty_like(X)
    fn = (L.load().silhouette_sqeuclid_backward if metric == "sqeuclid"
          else L.load().silhouette_cosine_backward)
    rc = fn(_ptr(X), L.SIL_F32, None, _ptr(labels), N, D, int(K), flags, _ptr(gS), _ptr(dX),
            _ptr(workspace), workspace.numel(), _stream(X.device))
    L.check(rc, f"silhouette_{metric}_backward")
    return dX


class SilhouetteFn(torch.autograd.Function):
    """S = Silhouette(X, labels) as a differentiable function of X (labels held fixed).

    Forward and backward both run in the HIP library; the workspace of the forward call (with
    a_i, b_i and the neighbouring cluster of every point) is kept for the backward.
    """

    @staticmethod
    def forward(ctx, X, labels, K, metric="sqeuclid", centre=True):
        X = X.contiguous()
        N, D = X.shape
        flags = (0 if centre else L.SIL_FLAG_NO_CENTRE) | L.SIL_FLAG_SAVE_FOR_GRAD
        ws = new_workspace(N, D, K, metric, X.dtype, flags, X.device)
        _, S = silhouette(X, labels, K, metric, centre=centre, want_s=False, save_for_grad=True,
                          workspace=ws)
        ctx.save_for_backward(X, labels, ws)
        ctx.K, ctx.metric, ctx.centre = K, metric, centre
        return S

    @staticmethod
    def backward(ctx, grad_S):
        X, labels, ws = ctx.saved_tensors
        dX = silhouette_backward(X, labels, ctx.K, ctx.metric, grad_S, ws, centre=ctx.centre)
        return dX, None, None, None, None


class BatchedSilhouette:
    """Many problems (for instance the labelings of a k-sweep) evaluated together.

    problems: a list of (X, labels, K, metric) with X float32 [N, D] (D <= 128) and labels int32
    [N] on one GPU.  Results land in ``self.S`` (float64 [len(problems)]) and, with want_s,
    ``self.s[i]`` (float32 [N_i]).  The workspace is allocated here once and owned by the plan.
    """

    def __init__(self, problems, *, want_s: bool = True, centre: bool = True,
                 euclid_approx: bool = False):
        if not problems:
            raise ValueError("no problems")
        dev = problems[0][0].device
        self.device = dev
        self.problems = problems
        self.S = torch.full((len(problems),), float("nan"), dtype=torch.float64, device=dev)
        self.s = []
        arr = (L.SilProblem * len(problems))()
        for i, (X, labels, K, metric) in enumerate(problems):
            _check_inputs(X, labels, None)
            if X.dtype != torch.float32:
                raise TypeError("batched problems take float32 X")
            s = torch.empty(X.shape[0], dtype=torch.float32, device=dev) if want_s else None
            self.s.append(s)
            arr[i] = L.SilProblem(X.data_ptr(), labels.data_ptr(), X.shape[0], X.shape[1], int(K),
                                  L.SIL_F32, METRIC[metric], 0 if s is None else s.data_ptr(),
                                  self.S.data_ptr() + 8 * i)
        self._arr = arr
        plan = ctypes.c_void_p()
        lib = L.load()
        flags = (0 if centre else L.SIL_FLAG_NO_CENTRE) | (L.SIL_FLAG_EUCLID_APPROX if euclid_approx else 0)
        self.flags = flags
        self.tuned_from_cache = False
        L.check(lib.silhouette_batched_plan(arr, len(problems), flags, ctypes.byref(plan)),
                "silhouette_batched_plan")
        self._plan = plan
        self.workspace = torch.empty(lib.silhouette_batched_workspace_bytes(plan), dtype=torch.uint8,
                                     device=dev)

    def _ws(self):
        return _ptr(self.workspace), self.workspace.numel()

    def run(self, stream: Optional[torch.cuda.Stream] = None):
        st = ctypes.c_void_p((stream or torch.cuda.current_stream(self.device)).cuda_stream)
        L.check(L.load().silhouette_batched_run(self._plan, *self._ws(), st), "silhouette_batched_run")
        return self.S

    def tune_key(self):
        """(key, shape) of this plan in the tuner's cache (see tune_cache.plan_key)."""
        from .tune_cache import plan_key
        props = torch.cuda.get_device_properties(self.device)
        return plan_key(props.gcnArchName, props.multi_processor_count, "f32", self.flags,
                        [(m, X.shape[0], X.shape[1], K) for X, _, K, m in self.problems])

    def tune(self, cache=None) -> float:
        """Autotune the persistent launch on these problems; returns its time in ms.

        cache (a path or a tune_cache.TuneCache): a plan whose signature is in the cache takes the
        stored configuration without timing any launch (``self.tuned_from_cache`` is then True and
        the stored time is returned); otherwise the tuner's choice is stored there."""
        from .tune_cache import TuneCache
        if isinstance(cache, (str, os.PathLike)):
            cache = TuneCache(os.fspath(cache))
        key = shape = None
        if cache is not None:
            key, shape = self.tune_key()
            hit = cache.get(key)
            if hit is not None:
                self.set_config(**hit["config"])
                self.run()  # as after tuning: statistics, tables and results in the workspace
                self.tuned_from_cache = True
                return hit["ms"]
        ms = ctypes.c_float()
        L.check(L.load().silhouette_batched_tune(self._plan, *self._ws(), _stream(self.device),
                                                 ctypes.byref(ms)), "silhouette_batched_tune")
        self.tuned_from_cache = False
        if cache is not None:
            cache.put(key, self.config(), ms.value, shape)
        return ms.value

    def config(self) -> dict:
        out = (ctypes.c_int32 * 7)()
        L.check(L.load().silhouette_batched_config(self._plan, out, 7), "silhouette_batched_config")
        return {"grid": out[0], "grab": out[1], "order": ("cost", "problem")[out[2]],
                "rows_per_item": {16: 128 * out[3], 24: 128 * out[4], 32: 128 * out[5]},
                "share_x": bool(out[6])}

    def set_config(self, grid: int, grab: int = 1, order: str = "cost", rows_per_item=None,
                   share_x: bool = True):
        """Pin the launch configuration (rows_per_item: {16|24|32: 128 or 256}, keyed by GEMM depth;
        share_x: problems with the same X, D and metric read their rows once for all of them)."""
        rpi = {16: 128, 24: 128, 32: 128, **(rows_per_item or {})}
        cfg = (ctypes.c_int32 * 7)(grid, grab, {"cost": 0, "problem": 1}[order], rpi[16] // 128,
                                   rpi[24] // 128, rpi[32] // 128, int(bool(share_x)))
        L.check(L.load().silhouette_batched_set_config(self._plan, cfg, 7), "silhouette_batched_set_config")

    def capture(self, stream: torch.cuda.Stream):
        """Capture one run into a hipGraph on `stream` (a non-default stream)."""
        L.check(L.load().silhouette_batched_capture(self._plan, *self._ws(),
                                                    ctypes.c_void_p(stream.cuda_stream)),
                "silhouette_batched_capture")

    def replay(self, stream: Optional[torch.cuda.Stream] = None):
        st = ctypes.c_void_p((stream or torch.cuda.current_stream(self.device)).cuda_stream)
        L.check(L.load().silhouette_batched_replay(self._plan, st), "silhouette_batched_replay")
        return self.S

    def status(self):
        """Per-problem device status (list of sil_status codes); waits for the current stream."""
        out = (ctypes.c_int32 * len(self.problems))()
        L.load().silhouette_batched_status(self._plan, _ptr(self.workspace), out, _stream(self.device))
        return list(out)

    def close(self):
        if getattr(self, "_plan", None):
            L.load().silhouette_batched_free(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
