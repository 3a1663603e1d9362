"""Mahalanobis Silhouette on the GPU (transform on fp32 MFMA, then the fp32 squared Euclidean
path) against the FP64 oracle, which works with M = L^T L directly and never forms L x.  The
per-point bound is the fp32 form's bound on Z = X L^T (formed here in binary64) plus the
transform's fp32 rounding carried through a_i and b_i."""

import numpy as np
import pytest
import torch

import oracle
from paper_2303_14102_amd import workloads as wl
from parity_helpers import U32, dequantised, per_point_bound, storage

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_14102_amd import _lib
    _lib.load()  # fails loudly when the library is missing
    return torch.device("cuda:0")


def mahal_bound(Xh, Lh, labels, K, a, b):
    Xh = np.asarray(Xh, np.float64)
    D = Xh.shape[1]
    Z = Xh @ Lh.T
    base = per_point_bound("f32", 0, "sqeuclid", True, Z, labels, K, a, b)
    # |z~ - z| per element <= (D + 4) u sum_k |L_ck x_k|; the cluster means move by at most the
    # largest row error
    e = (D + 4) * U32 * np.sqrt(((np.abs(Xh) @ np.abs(Lh).T) ** 2).sum(axis=1))
    et = e + e.max()
    da = 2 * (2 * np.sqrt(np.abs(a)) * et + et ** 2)  # a carries N_o / (N_o - 1) <= 2
    db = 2 * np.sqrt(np.abs(b)) * et + et ** 2
    return base + 2 * (da + db) / np.maximum(np.maximum(a, b), 1e-30)


def make_L(D, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "full":
        L = rng.standard_normal((D, D)) / np.sqrt(D) + np.eye(D)
    elif kind == "rank":  # half the rows zero: M = L^T L has rank D / 2
        L = rng.standard_normal((D, D)) / np.sqrt(D)
        L[D // 2:] = 0.0
    else:
        L = np.diag(rng.uniform(0.2, 3.0, size=D))
    return np.ascontiguousarray(L, dtype=np.float32)


CASES = [
    # (N, D, K, form, L kind, singletons, seed)
    (5_037, 40, 70, "f32", "full", 2, 1),
    (3_001, 128, 100, "bf16", "full", 1, 2),
    (2_000, 256, 40, "f32", "rank", 0, 3),
    (4_099, 16, 33, "fp8", "diag", 1, 4),
    (1_500, 3, 5, "f32", "full", 1, 5),
    (120_001, 64, 200, "bf16", "full", 0, 6),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c[0]}-D{c[1]}-K{c[2]}-{c[3]}-{c[4]}")
def test_mahalanobis_parity(dev, case):
    from paper_2303_14102_amd import binding as sil
    n, d, k, form, kind, single, seed = case
    b = wl.make_small(n, d, k, seed=seed, singletons=single)
    Xd, sc, codes = storage(b.X.to(dev), form)
    Lh = make_L(d, kind, seed)
    print(f"[mahal] N={n} D={d} K={k} form={form} L={kind}", flush=True)
    s, S = sil.silhouette_mahalanobis(Xd, b.labels.to(dev), k, torch.from_numpy(Lh).to(dev), col_scale=sc,
                                      check_status=True)
    cs = None if sc is None else sc.cpu().numpy()
    Xh = dequantised(codes, cs)
    M = Lh.astype(np.float64).T @ Lh.astype(np.float64)
    s_ref, S_ref, a, bb = oracle.silhouette_mahalanobis(codes, b.labels.numpy(), k, M, col_scale=cs,
                                                        details=True)
    bound = mahal_bound(Xh, Lh.astype(np.float64), b.labels.numpy(), k, a, bb)
    ds = np.abs(s.cpu().numpy().astype(np.float64) - s_ref)
    print(f"  S={S.item():.10f} ref={S_ref:.10f} max|ds|={ds.max():.2e} max(|ds|/bound)={(ds / bound).max():.3f}",
          flush=True)
    assert np.all(ds <= bound)
    assert abs(S.item() - S_ref) <= max(1e-6, bound.mean())


def test_identity_matches_squared_euclidean(dev):
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(20_011, 40, 70, seed=7, singletons=2)
    X, lab = b.X.to(dev), b.labels.to(dev)
    s1, S1 = sil.silhouette_mahalanobis(X, lab, 70, torch.eye(40, device=dev), check_status=True)
    s2, S2 = sil.silhouette(X, lab, 70, check_status=True)
    # X I^T is exact on the MFMA; the FP64 cluster sums may differ in the order of rows within a
    # cluster (the counting sort's)
    assert float((s1 - s2).abs().max()) <= 1e-6 and abs(S1.item() - S2.item()) <= 1e-12


def test_nonfinite_L_is_a_data_error(dev):
    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(2_000, 8, 4, seed=8)
    L = torch.eye(8, device=dev)
    L[3, 5] = float("nan")
    with pytest.raises(_lib.SilhouetteError) as e:
        sil.silhouette_mahalanobis(b.X.to(dev), b.labels.to(dev), 4, L, check_status=True)
    assert e.value.code == -6
