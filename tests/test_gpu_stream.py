"""Out-of-core evaluation (X and labels in host memory, streamed in chunks): equal to the
in-memory call on the same data up to the order of the FP64 cluster sums, and to the FP64 oracle
within the per-point bound; chunks holding a single cluster, pageable host memory, errors found
in a late chunk, and a workspace reused across calls."""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_2303_14102_amd import workloads as wl
from parity_helpers import TOL_S_MEAN, dequantised, per_point_bound, storage

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_14102_amd import _lib
    _lib.load()  # fails loudly when the library is missing
    return torch.device("cuda:0")


def host_copy(Xd):
    return Xd.cpu().contiguous().pin_memory()


CASES = [
    # (N, D, K, metric, form, chunk_rows, approx, seed, products)
    (20_011, 40, 70, "sqeuclid", "f32", 4_097, False, 1, 0),
    (20_011, 40, 70, "cosine", "bf16", 1_000, False, 2, 0),
    (9_999, 128, 100, "sqeuclid", "bf16", 9_999, False, 3, 0),
    (9_999, 128, 100, "sqeuclid", "bf16", 50_000, False, 4, 0),
    (12_345, 16, 33, "sqeuclid", "fp8", 3_000, False, 5, 0),
    (15_000, 64, 50, "sqeuclid", "f32", 2_048, True, 6, 0),
    (150_001, 64, 300, "sqeuclid", "bf16", 40_000, False, 7, 0),
    # two products on the exact x: the folded centring uses the whole data set's mean
    (40_003, 128, 200, "sqeuclid", "bf16", 10_000, False, 8, 2),
    (40_003, 128, 200, "cosine", "bf16", 12_000, False, 9, 2),
    (30_011, 128, 150, "sqeuclid", "fp8", 8_000, False, 10, 2),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c[0]}-D{c[1]}-{c[3]}-{c[4]}-c{c[5]}-P{c[8]}{'-approx' if c[6] else ''}")
def test_stream_equals_in_memory(dev, case):
    from paper_2303_14102_amd import binding as sil
    n, d, k, metric, form, chunk, approx, seed, products = case
    b = wl.make_small(n, d, k, seed=seed, singletons=1)
    Xd, sc, codes = storage(b.X.to(dev), form)
    lab_d = b.labels.to(dev)
    print(f"[stream] {case}", flush=True)
    # the streamed chunks run the two-product sweep itself (not the in-memory form's screen)
    s_mem, S_mem = sil.silhouette(Xd, lab_d, k, metric, products=products, col_scale=sc,
                                  euclid_approx=approx, screen=False, check_status=True)
    s_st, S_st = sil.silhouette_stream(host_copy(Xd), b.labels.contiguous().pin_memory(), k, metric,
                                       chunk_rows=chunk, products=products, col_scale=sc,
                                       euclid_approx=approx, device=dev, check_status=True)
    dmax = float((s_st - s_mem.cpu()).abs().max())
    print(f"  S_mem={S_mem.item():.12f} S_stream={S_st.item():.12f} max|ds|={dmax:.2e}", flush=True)
    assert dmax <= 2e-6
    assert abs(S_st.item() - S_mem.item()) <= 1e-9
    # and the oracle, on the streamed result
    m = "euclid_approx" if approx else metric
    cs = None if sc is None else sc.cpu().numpy()
    s_ref, S_ref, a, bb, _ = oracle.silhouette(codes, b.labels.numpy(), k, m, col_scale=cs, details=True)
    bound = per_point_bound(form, (products or 3) if form != "f32" else 0, m, True, dequantised(codes, cs),
                            b.labels.numpy(), k, a, bb)
    assert np.all(np.abs(s_st.numpy().astype(np.float64) - s_ref) <= bound)
    assert abs(S_st.item() - S_ref) <= TOL_S_MEAN[form]


def test_stream_chunks_of_one_cluster(dev):
    # rows sorted by label: most chunks hold a single cluster, which is no error for a chunk
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(30_000, 24, 6, seed=8)
    order = torch.argsort(b.labels, stable=True)
    X, lab = b.X[order].contiguous(), b.labels[order].contiguous()
    s_mem, S_mem = sil.silhouette(X.to(dev), lab.to(dev), 6, check_status=True)
    s_st, S_st = sil.silhouette_stream(X.pin_memory(), lab.pin_memory(), 6, chunk_rows=1_500, device=dev,
                                       check_status=True)
    assert float((s_st - s_mem.cpu()).abs().max()) <= 2e-6
    assert abs(S_st.item() - S_mem.item()) <= 1e-9


def test_stream_pageable_host_memory(dev):
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(10_007, 32, 20, seed=9)
    s_mem, S_mem = sil.silhouette(b.X.to(dev), b.labels.to(dev), 20, check_status=True)
    s_st, S_st = sil.silhouette_stream(b.X.contiguous(), b.labels.contiguous(), 20, chunk_rows=3_333,
                                       device=dev, check_status=True)
    assert float((s_st - s_mem.cpu()).abs().max()) <= 2e-6
    assert abs(S_st.item() - S_mem.item()) <= 1e-9


def test_stream_errors(dev):
    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(12_000, 16, 5, seed=10)
    lab = b.labels.clone()
    lab[11_990] = 5  # outside [0, K), in the last chunk
    with pytest.raises(_lib.SilhouetteError) as e:
        sil.silhouette_stream(b.X.pin_memory(), lab.pin_memory(), 5, chunk_rows=4_000, device=dev,
                              check_status=True)
    assert e.value.code == -3
    s, S = sil.silhouette_stream(b.X.pin_memory(), lab.pin_memory(), 5, chunk_rows=4_000, device=dev)
    assert math.isnan(S.item()) and torch.isnan(s).all()
    one = torch.zeros(12_000, dtype=torch.int32)
    with pytest.raises(_lib.SilhouetteError) as e:
        sil.silhouette_stream(b.X.pin_memory(), one.pin_memory(), 5, chunk_rows=4_000, device=dev,
                              check_status=True)
    assert e.value.code == -4
    ws = torch.empty(sil.stream_workspace_bytes(12_000, 4_000, 16, 5), dtype=torch.uint8, device=dev)
    with pytest.raises(_lib.SilhouetteError) as e:  # the library's own check of the chunk size
        sil.silhouette_stream(b.X.pin_memory(), b.labels.pin_memory(), 5, chunk_rows=0, workspace=ws,
                              device=dev)
    assert e.value.code == -1


def test_stream_workspace_reused(dev):
    from paper_2303_14102_amd import binding as sil
    ws = torch.empty(sil.stream_workspace_bytes(20_000, 3_000, 24, 12), dtype=torch.uint8, device=dev)
    for seed in (11, 12):
        b = wl.make_small(20_000, 24, 12, seed=seed)
        s_mem, S_mem = sil.silhouette(b.X.to(dev), b.labels.to(dev), 12, check_status=True)
        s_st, S_st = sil.silhouette_stream(b.X.pin_memory(), b.labels.pin_memory(), 12, chunk_rows=3_000,
                                           workspace=ws, device=dev, check_status=True)
        assert abs(S_st.item() - S_mem.item()) <= 1e-9
        assert float((s_st - s_mem.cpu()).abs().max()) <= 2e-6
