"""Shared pieces of the GPU parity tests: the per-point error bound of the kernel's arithmetic
and the storage conversions.

Per-point bound: with the cross term x'.mu'_k carried to a relative accuracy eps (fp32
accumulation over D terms, or the bf16 hi/lo split with 1, 2 or 3 products),
|db_i| <= 2 eps ||x'_i|| max_k ||mu'_k|| plus fp32 rounding of ||x'_i||^2 + c_k; a_i comes from
the difference form in fp32; then |ds_i| <= 2 (|da_i| + |db_i|) / max(a_i, b_i).
"""

import numpy as np
import torch

from paper_2303_14102_amd import workloads as wl

TOL_S_MEAN = {"f32": 1e-6, "bf16": 1e-4, "fp8": 1e-4}
U32 = 2.0 ** -24


def cross_term_eps(form, products, metric, centre, D):
    """Relative accuracy of the computed cross term x'.mu'_k."""
    acc = U32 * (D + 8)                      # fp32 accumulation (MFMA or the epilogue)
    if form == "f32":
        return acc
    exact_x = metric == "sqeuclid" and not centre  # bf16/fp8 storage is exact in bf16 uncentred
    if products == 2 and form in ("bf16", "fp8") and metric in ("sqeuclid", "cosine"):
        # x itself enters the GEMM (fp8: its codes, the tables carrying the column scales): the
        # folded centring (squared Euclidean, the bound then uses |x|), or the cosine form scaled
        # by 1 / |x| after the minimum (relative to |z| = 1)
        exact_x = True
    mu_split = 2.0 ** -16                    # hi + lo carries ~16 bits of the mean
    if products == 3:
        return 2.0 ** -16 + acc
    if products == 2:
        return (mu_split if exact_x else 2.0 ** -8) + acc
    return 2.0 ** -8 + (0.0 if exact_x else 2.0 ** -8) + acc


def bound_from_stats(form, products, metric, centre, rows, stats, a, b, root=False):
    """Bound on |s_i(GPU) - s_i(oracle)| for the given rows (binary64 values as stored), from
    binary64 cluster statistics (count, V, psi) of the whole data set.  root: the approximate
    Euclidean form, where a and b (the oracle's, already square roots) are roots of the mean
    squared distances: the squared quantities' error bounds pass through the square root as
    interval widths."""
    count, V, psi = stats
    rows = np.asarray(rows, np.float64)
    D = rows.shape[1]
    cnt = np.asarray(count, np.float64)
    ne = cnt > 0
    mu = V[ne] / cnt[ne, None]
    if metric == "sqeuclid":
        m = V.sum(0) / cnt.sum() if centre else np.zeros(D)
        xp = rows - m
        mup = mu - m
        var = psi[ne] / cnt[ne] - (mu * mu).sum(1)
        cmax = ((mup * mup).sum(1) + var).max()
    else:
        xp = rows / np.linalg.norm(rows, axis=1, keepdims=True)
        mup = mu
        cmax = 1.0
    nx = np.linalg.norm(xp, axis=1)
    eps = cross_term_eps(form, products, metric, centre, D)
    nxc = nx  # norm of the GEMM operand
    if metric == "sqeuclid" and centre and form in ("bf16", "fp8") and products == 2:
        # folded centring: the GEMM multiplies x itself, and c_k carries 2 m.mu'_k
        nxc = np.linalg.norm(rows, axis=1)
        cmax = cmax + 2 * np.abs(mup @ m).max()
    if root:  # the squared quantities and their bounds, then the roots' interval widths
        a2, b2 = np.asarray(a) ** 2, np.asarray(b) ** 2
        db2 = 2 * eps * nxc * np.linalg.norm(mup, axis=1).max() + 4 * U32 * (nx ** 2 + nxc ** 2 + cmax)
        da2 = 4 * U32 * (D + 8) * (a2 + np.abs(a2))
        da = np.sqrt(a2 + da2) - np.sqrt(np.maximum(a2 - da2, 0.0))
        db = np.sqrt(b2 + db2) - np.sqrt(np.maximum(b2 - db2, 0.0))
        return 2 * (da + db) / np.maximum(np.maximum(a, b), 1e-30) + 4 * U32
    db = 2 * eps * nxc * np.linalg.norm(mup, axis=1).max() + 4 * U32 * (nx ** 2 + nxc ** 2 + cmax)
    da = 4 * U32 * (D + 8) * (a + np.abs(a))
    return 2 * (da + db) / np.maximum(np.maximum(a, b), 1e-30) + 4 * U32


def sqeuclid_bounds_all_rows(form, products_list, codes, cs, stats, a, b, chunk=1 << 21):
    """bound_from_stats for the centred squared Euclidean forms over every row of a large data
    set, for several product counts at once: the two row norms it needs (|x - m| and |x|) are
    formed a chunk at a time with torch on the host, in binary64."""
    count, V, psi = stats
    cnt = np.asarray(count, np.float64)
    ne = cnt > 0
    mu = V[ne] / cnt[ne, None]
    m = V.sum(0) / cnt.sum()
    mup = mu - m
    var = psi[ne] / cnt[ne] - (mu * mu).sum(1)
    cmax0 = ((mup * mup).sum(1) + var).max()
    mupmax = np.linalg.norm(mup, axis=1).max()
    D = V.shape[1]
    N = len(a)
    nx = np.empty(N)
    nxc = np.empty(N)
    mt = torch.from_numpy(m)
    for i0 in range(0, N, chunk):
        i1 = min(N, i0 + chunk)
        rows = torch.from_numpy(np.ascontiguousarray(dequantised(codes[i0:i1], cs))).double()
        nxc[i0:i1] = torch.linalg.vector_norm(rows, dim=1).numpy()
        nx[i0:i1] = torch.linalg.vector_norm(rows - mt, dim=1).numpy()
    a = np.asarray(a)
    b = np.asarray(b)
    da = 4 * U32 * (D + 8) * (a + np.abs(a))
    den = np.maximum(np.maximum(a, b), 1e-30)
    out = {}
    for products in products_list:
        eps = cross_term_eps(form, products, "sqeuclid", True, D)
        folded = form in ("bf16", "fp8") and products == 2
        ng = nxc if folded else nx  # norm of the GEMM operand
        cmax = cmax0 + (2 * np.abs(mup @ m).max() if folded else 0.0)
        db = 2 * eps * ng * mupmax + 4 * U32 * (nx ** 2 + ng ** 2 + cmax)
        out[products] = 2 * (da + db) / den + 4 * U32
    return out


def plain_stats(X, labels, K, metric):
    metric = "sqeuclid" if metric == "euclid_approx" else metric
    """count, V, psi of a small data set with numpy (for the bound only)."""
    X = np.asarray(X, np.float64)
    cnt = np.bincount(labels, minlength=K)
    V = np.zeros((K, X.shape[1]))
    np.add.at(V, labels, X if metric == "sqeuclid" else X / np.linalg.norm(X, axis=1, keepdims=True))
    psi = np.zeros(K)
    if metric == "sqeuclid":
        np.add.at(psi, labels, (X * X).sum(1))
    return cnt, V, psi


def per_point_bound(form, products, metric, centre, Xh, labels, K, a, b):
    """Per-point bound for every row of a small data set (metric may be euclid_approx)."""
    root = metric == "euclid_approx"
    m = "sqeuclid" if root else metric
    return bound_from_stats(form, products, m, centre, Xh, plain_stats(Xh, labels, K, m), a, b, root)


def dequantised(codes, col_scale):
    if codes.dtype == np.uint16:
        return (codes.astype(np.uint32) << 16).view(np.float32)
    if codes.dtype == np.uint8:
        return torch.from_numpy(np.ascontiguousarray(codes)).view(torch.float8_e4m3fn).float().numpy() * col_scale
    return codes


def storage(X32: torch.Tensor, form: str):
    """(X on device in the given storage, col_scale or None, host codes for the oracle)."""
    if form == "f32":
        return X32, None, wl.host_codes(X32)
    if form == "bf16":
        q = wl.to_bf16(X32)
        return q, None, wl.host_codes(q)
    q, sc = wl.to_fp8_e4m3(X32)
    return q, sc, wl.host_codes(q)


def kmeans_dist_bound(form, centre, X, labels, K, products=3):
    """Per-point bound on |d~(x_i, mu_k) - d(x_i, mu_k)| for the K-means assignment's squared
    distance ||x'||^2 + ||mu'_k||^2 - 2 x'.mu'_k, formed like the Silhouette's b-path (cross term
    to relative accuracy eps, fp32 rounding of the sum), with the means of the given labels.
    products = 2 with bf16 storage: the folded centring (the cross term multiplies x itself and
    the constant carries 2 m.mu'_k)."""
    X = np.asarray(X, np.float64)
    D = X.shape[1]
    ids = np.unique(labels)
    mu = np.stack([X[labels == k].mean(axis=0) for k in ids])
    m = X.mean(axis=0) if centre else np.zeros(D)
    xp, mup = X - m, mu - m
    nx = np.linalg.norm(xp, axis=1)
    nmu = np.linalg.norm(mup, axis=1)
    eps = cross_term_eps(form, products, "sqeuclid", centre, D)
    cmax = (nmu ** 2).max()
    nxc = nx
    if form == "bf16" and products == 2 and centre:
        nxc = np.linalg.norm(X, axis=1)
        cmax = cmax + 2 * np.abs(mup @ m).max()
    return 2 * eps * nxc * nmu.max() + 4 * U32 * (nx ** 2 + nxc ** 2 + cmax)
