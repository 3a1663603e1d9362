"""Generalized Kullback-Leibler Silhouette on the GPU against the FP64 oracle: positive data
(exponentiated Gaussian blobs), fp32 and bf16 storage, several split-product forms, ragged shapes,
singletons; the domain error; invariance to scaling the data."""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_2303_14102_amd import workloads as wl
from parity_helpers import TOL_S_MEAN, U32, cross_term_eps, dequantised, storage

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_14102_amd import _lib
    _lib.load()  # fails loudly when the library is missing
    return torch.device("cuda:0")


def kl_bound(form, products, X, labels, K, a, b):
    """Per-point bound on |s_i(GPU) - s_i(oracle)|: the row term phi(x) in fp32 (logf, D terms),
    the cross term x . (mean log y) to relative accuracy eps, the statistics' per-entry log in
    fp32 (relative 4 u32 of |log y|, summed in FP64), and fp32 rounding of c_k and of the sums;
    the a-path's fp32 dot product; self-exclusion scales a by at most 2."""
    X = np.asarray(X, np.float64)
    D = X.shape[1]
    cnt = np.bincount(labels, minlength=K)
    G = np.zeros((K, D))
    np.add.at(G, labels, np.log(X))
    A = np.zeros((K, D))
    np.add.at(A, labels, np.abs(np.log(X)))
    ne = cnt > 0
    g = G[ne] / cnt[ne, None]
    amax = np.linalg.norm(A[ne] / cnt[ne, None], axis=1).max()
    c = np.zeros(K)
    np.add.at(c, labels, X.sum(1))
    c = c[ne] / cnt[ne]
    nx = np.linalg.norm(X, axis=1)
    gmax = np.linalg.norm(g, axis=1).max()
    phi_abs = (np.abs(X * np.log(X)) + X).sum(1)
    eps = cross_term_eps(form, products, "sqeuclid", False, D) + U32
    dA = (D + 8) * U32 * phi_abs
    sums = 3 * U32 * (phi_abs + np.abs(c).max() + nx * gmax)
    lg = 4 * U32 * nx * amax
    db = dA + eps * nx * gmax + lg + sums
    da = 2 * (dA + (D + 4) * U32 * nx * gmax + lg + sums)
    return 2 * (da + db) / np.maximum(np.maximum(a, b), 1e-30) + 4 * U32


def positive_blobs(n, d, k, seed, single):
    b = wl.make_small(n, d, k, seed=seed, singletons=single)
    return torch.exp(b.X / 4.0), b.labels


CASES = [
    # (N, D, K, form, products, singletons, seed)
    (5_037, 40, 70, "f32", 0, 2, 1),
    (3_001, 128, 100, "bf16", 3, 1, 2),
    (4_099, 16, 33, "bf16", 2, 1, 3),
    (2_000, 256, 40, "f32", 0, 0, 4),
    (1_500, 3, 5, "bf16", 1, 1, 5),
    (140_001, 64, 300, "bf16", 3, 0, 6),
    (60_001, 128, 257, "f32", 0, 1, 9),   # whole-wave row statistics, 512-byte rows
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c[0]}-D{c[1]}-K{c[2]}-{c[3]}-P{c[4]}")
def test_kl_parity(dev, case):
    from paper_2303_14102_amd import binding as sil
    n, d, k, form, products, single, seed = case
    X, lab = positive_blobs(n, d, k, seed, single)
    Xd, sc, codes = storage(X.to(dev), form)
    print(f"[kl] N={n} D={d} K={k} form={form} P={products}", flush=True)
    s, S = sil.silhouette(Xd, lab.to(dev), k, "kl", products=products, check_status=True)
    lab_h = lab.numpy()
    s_ref, S_ref, a, bb, _ = oracle.silhouette(codes, lab_h, k, "kl", details=True)
    bound = kl_bound(form, products, dequantised(codes, None), lab_h, k, a, bb)
    ds = np.abs(s.cpu().numpy().astype(np.float64) - s_ref)
    print(f"  S={S.item():.10f} ref={S_ref:.10f} max|ds|={ds.max():.2e} max(|ds|/bound)={(ds / bound).max():.3f}",
          flush=True)
    assert np.all(ds <= bound)
    tol = TOL_S_MEAN[form] if products in (0, 3) else max(TOL_S_MEAN[form], bound.mean())
    assert abs(S.item() - S_ref) <= tol


def test_kl_scale_invariance(dev):
    # d(cx, cy) = c d(x, y), so s is unchanged when the data are scaled
    from paper_2303_14102_amd import binding as sil
    X, lab = positive_blobs(20_011, 24, 40, 7, 1)
    s1, S1 = sil.silhouette(X.to(dev), lab.to(dev), 40, "kl", check_status=True)
    s2, S2 = sil.silhouette((8.0 * X).to(dev), lab.to(dev), 40, "kl", check_status=True)
    assert float((s1 - s2).abs().max()) <= 1e-4 and abs(S1.item() - S2.item()) <= 1e-6


@pytest.mark.parametrize("d,form", [(16, "f32"), (128, "bf16"), (64, "f32")])
def test_kl_domain_error(dev, d, form):
    # a zero entry: chunked statistics (D = 16) and whole-wave rows (256-byte rows)
    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    X, lab = positive_blobs(3_000, d, 6, 8, 0)
    X[1_234, 5] = 0.0
    Xd = storage(X.to(dev), form)[0]
    with pytest.raises(_lib.SilhouetteError) as e:
        sil.silhouette(Xd, lab.to(dev), 6, "kl", check_status=True)
    assert e.value.code == -9
    s, S = sil.silhouette(Xd, lab.to(dev), 6, "kl")
    assert math.isnan(S.item()) and torch.isnan(s).all()
