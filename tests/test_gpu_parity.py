"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same seeded inputs.

Tolerances:
  - cluster sizes: exact;  Y / Omega / Psi: relative 1e-12 (FP64 sums in another order);
  - S: |dS| <= 1e-6 for fp32 storage, <= 1e-4 for bf16 / fp8 storage (oracle on the dequantised
    input);
  - s_i: the error bound of the kernel's arithmetic, per point (parity_helpers.per_point_bound).
"""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_2303_14102_amd import workloads as wl
from parity_helpers import TOL_S_MEAN, U32, dequantised, per_point_bound, storage  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_14102_amd import _lib
    _lib.load()  # fails loudly when the library is missing
    return torch.device("cuda:0")


def run_case(dev, X32, labels, K, metric, form, products=0, centre=True):
    from paper_2303_14102_amd import binding as sil
    Xd, sc, codes = storage(X32.to(dev), form)
    lab = labels.to(dev)
    print(f"[case] N={X32.shape[0]} D={X32.shape[1]} K={K} metric={metric} form={form} "
          f"products={products} centre={centre}", flush=True)
    s, S = sil.silhouette(Xd, lab, K, metric, products=products, centre=centre, col_scale=sc,
                          check_status=True)
    torch.cuda.synchronize()
    cs = None if sc is None else sc.cpu().numpy()
    lab_h = labels.cpu().numpy()
    s_ref, S_ref, a, b, _ = oracle.silhouette(codes, lab_h, K, metric, col_scale=cs, details=True)
    bound = per_point_bound(form, products, metric, centre, dequantised(codes, cs), lab_h, K, a, b)
    s = s.cpu().numpy().astype(np.float64)
    worst = np.abs(s - s_ref) / bound
    print(f"  S={S.item():.10f} ref={S_ref:.10f} |dS|={abs(S.item() - S_ref):.2e} "
          f"max|ds|={np.abs(s - s_ref).max():.2e} max(|ds|/bound)={worst.max():.3f}", flush=True)
    assert np.all(np.abs(s - s_ref) <= bound), f"point {int(worst.argmax())} exceeds its bound"
    # S is the mean of s_i: the reduced forms (1 or 2 products on a split point) are held to the
    # mean of their per-point bounds, the full forms to the stated targets
    tol_S = TOL_S_MEAN[form] if products in (0, 3) else max(TOL_S_MEAN[form], bound.mean())
    assert abs(S.item() - S_ref) <= tol_S
    return s, S.item(), s_ref, S_ref


# ---------------------------------------------------------------------------------------------
# cluster statistics


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
@pytest.mark.parametrize("form", ["f32", "bf16", "fp8"])
def test_stats_parity(dev, metric, form):
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(20_011, 40, 70, seed=3, singletons=2)  # ragged everywhere, 5 segments
    Xd, sc, codes = storage(b.X.to(dev), form)
    print(f"[stats] metric={metric} form={form}", flush=True)
    count, V, psi = sil.cluster_stats(Xd, b.labels.to(dev), 73, metric, col_scale=sc)
    c_ref, V_ref, p_ref = oracle.cluster_stats(codes, b.labels.numpy(), 73, metric,
                                               col_scale=None if sc is None else sc.cpu().numpy())
    assert np.array_equal(count.cpu().numpy(), c_ref)
    scale = np.abs(V_ref).max()
    np.testing.assert_allclose(V.cpu().numpy(), V_ref, rtol=1e-12, atol=1e-12 * scale)
    np.testing.assert_allclose(psi.cpu().numpy(), p_ref, rtol=1e-12, atol=0)


# statistics of rows of 256, 512 or 1024 bytes (the whole-wave row reduction; for cosine the
# batch's row norms are reduced across the wave together)
ROW_CASES = [(128, "bf16"), (256, "bf16"), (64, "f32"), (128, "f32"), (256, "f32"), (128, "fp8"),
             (256, "fp8")]


def row_case_labels(rng):
    # cluster sizes that put run boundaries on segment borders (4096 positions), on batch borders
    # (16, 8 or 4 rows), one row either side of them, and runs shorter than a batch; then the
    # cluster ids are shuffled and the rows permuted
    sizes = [4096, 4080, 16, 1, 15, 8192, 3, 4093, 2, 1, 12000, 17, 4, 4, 4, 4, 9000, 5, 4095]
    sizes += list(rng.integers(1, 40, size=200)) + [0, 0, 7000]
    K = len(sizes)
    ids = rng.permutation(K)
    lab = np.repeat(ids, sizes).astype(np.int32)
    return lab[rng.permutation(len(lab))], K


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
@pytest.mark.parametrize("D,form", ROW_CASES, ids=lambda v: str(v))
def test_stats_row_reduction(dev, D, form, metric):
    from paper_2303_14102_amd import binding as sil
    rng = np.random.default_rng(D + len(form))
    lab, K = row_case_labels(rng)
    X = torch.from_numpy(rng.standard_normal((len(lab), D)).astype(np.float32) * 3 + 1)
    Xd, sc, codes = storage(X.to(dev), form)
    print(f"[stats-row] N={len(lab)} D={D} K={K} form={form} metric={metric}", flush=True)
    count, V, psi = sil.cluster_stats(Xd, torch.from_numpy(lab).to(dev), K, metric, col_scale=sc)
    c_ref, V_ref, p_ref = oracle.cluster_stats(codes, lab, K, metric,
                                               col_scale=None if sc is None else sc.cpu().numpy())
    assert np.array_equal(count.cpu().numpy(), c_ref)
    scale = np.abs(V_ref).max()
    np.testing.assert_allclose(V.cpu().numpy(), V_ref, rtol=1e-12, atol=1e-12 * scale)
    np.testing.assert_allclose(psi.cpu().numpy(), p_ref, rtol=1e-12, atol=0)


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
def test_stats_row_reduction_nonfinite(dev, metric):
    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(9_000, 128, 6, seed=9)
    X = b.X.clone()
    X[4321, 77] = float("inf")
    with pytest.raises(_lib.SilhouetteError) as e:
        sil.silhouette(X.to(dev).to(torch.bfloat16), b.labels.to(dev), 6, metric, check_status=True)
    assert e.value.code == -6


@pytest.mark.parametrize("D,form", [(128, "bf16"), (64, "f32"), (256, "f32"), (128, "fp8")])
def test_stats_row_reduction_zero_norm(dev, D, form):
    # a zero row in the middle of a batch, and one as the last row of the data
    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    for row in (5_003, 8_999):
        b = wl.make_small(9_000, D, 6, seed=10)
        X = b.X.clone()
        X[row] = 0.0
        Xd, sc, _ = storage(X.to(dev), form)
        with pytest.raises(_lib.SilhouetteError) as e:
            sil.silhouette(Xd, b.labels.to(dev), 6, "cosine", col_scale=sc, check_status=True)
        assert e.value.code == -5


@pytest.mark.parametrize("K", [4096, 4097, 9000])
def test_stats_scatter_forms(dev, K):
    # K <= 4096: the chunk is counting-sorted in LDS before the scatter; above: per-row placement
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(3 * K + 1_001, 12, K, seed=K, singletons=3)
    print(f"[stats-scatter] K={K}", flush=True)
    count, V, psi = sil.cluster_stats(b.X.to(dev), b.labels.to(dev), K)
    c_ref, V_ref, p_ref = oracle.cluster_stats(b.X.numpy(), b.labels.numpy(), K)
    assert np.array_equal(count.cpu().numpy(), c_ref)
    np.testing.assert_allclose(V.cpu().numpy(), V_ref, rtol=1e-12, atol=1e-12 * np.abs(V_ref).max())
    np.testing.assert_allclose(psi.cpu().numpy(), p_ref, rtol=1e-12, atol=0)


@pytest.mark.parametrize("K, offset_labels", [(600, False), (4096, True)])
def test_stats_large_chunk_sort(dev, K, offset_labels):
    # at least 256 chunks of 32768 labels and K >= 512: the histogram reads 64K-label chunks and
    # the scatter stages 32K-label chunks; labels that start 4 bytes past an aligned address take
    # the 4-byte loads instead of the 16-byte ones
    from paper_2303_14102_amd import binding as sil
    n = 256 * 32768 + 12_345
    b = wl.make_small(n, 4, K, seed=K + 1)
    lab = b.labels.to(dev)
    if offset_labels:
        buf = torch.empty(n + 1, dtype=torch.int32, device=dev)
        buf[1:] = lab
        lab = buf[1:]
        assert lab.data_ptr() % 16 == 4
    print(f"[stats-large-chunk] N={n} K={K} offset={offset_labels}", flush=True)
    count, V, psi = sil.cluster_stats(b.X.to(dev), lab, K)
    c_ref, V_ref, p_ref = oracle.cluster_stats(b.X.numpy(), b.labels.numpy(), K)
    assert np.array_equal(count.cpu().numpy(), c_ref)
    np.testing.assert_allclose(V.cpu().numpy(), V_ref, rtol=1e-11, atol=1e-11 * np.abs(V_ref).max())
    np.testing.assert_allclose(psi.cpu().numpy(), p_ref, rtol=1e-12, atol=0)


def test_stats_large_clusters_span_segments(dev):
    # a few clusters of ~1e5 points: every cluster crosses many segment borders
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(300_000, 24, 3, seed=8)
    count, V, psi = sil.cluster_stats(b.X.to(dev), b.labels.to(dev), 3)
    c_ref, V_ref, p_ref = oracle.cluster_stats(b.X.numpy(), b.labels.numpy(), 3)
    assert np.array_equal(count.cpu().numpy(), c_ref)
    np.testing.assert_allclose(V.cpu().numpy(), V_ref, rtol=1e-11, atol=1e-9)
    np.testing.assert_allclose(psi.cpu().numpy(), p_ref, rtol=1e-12)


# ---------------------------------------------------------------------------------------------
# the whole forward


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
def test_small_workload_fp32(dev, metric):
    b = wl.make_blobs(wl.WORKLOADS["blobs-10k-d8-k4"])
    s, S, s_ref, S_ref = run_case(dev, b.X, b.labels, 4, metric, "f32")
    assert abs(S - S_ref) <= TOL_S_MEAN["f32"]


CASES = [
    # (N, D, K, singletons, seed): several tiles of 32 clusters, ragged N / D / K, empty ids
    (5_037, 40, 70, 2, 11),
    (3_001, 128, 100, 1, 12),
    (2_000, 256, 40, 0, 13),
    (4_099, 16, 33, 1, 14),
    (1_500, 3, 5, 1, 15),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c[0]}-D{c[1]}-K{c[2]}")
@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
@pytest.mark.parametrize("form,products", [("f32", 0), ("bf16", 3), ("bf16", 2), ("bf16", 1),
                                           ("fp8", 3), ("fp8", 2)])
def test_forward_parity(dev, case, metric, form, products):
    N, D, K, single, seed = case
    b = wl.make_small(N, D, K, seed=seed, singletons=single, sigma=1.5)
    Kt = K + 2  # two unused ids
    s, S, s_ref, S_ref = run_case(dev, b.X, b.labels, Kt, metric, form, products)
    if form in ("bf16", "fp8") and products == 2:
        # x (fp8: its codes) enters the GEMM exact (folded centring; cosine scaled after the
        # minimum): the three-product form's accuracy on data near the origin
        assert abs(S - S_ref) <= TOL_S_MEAN[form]
    # singletons score exactly 0
    sizes = np.bincount(b.labels.numpy(), minlength=Kt)
    assert np.all(s[sizes[b.labels.numpy()] == 1] == 0.0)


# larger problems: ragged N over ~1000 workgroups, 4 to 16 cluster tiles, every precision form,
# many blocks that straddle a cluster boundary
LARGER_CASES = [
    # (N, D, K, metric, form, products, singletons, seed)
    (150_001, 64, 300, "sqeuclid", "bf16", 3, 1, 61),
    (140_333, 72, 257, "cosine", "bf16", 2, 0, 62),
    (131_200, 128, 400, "sqeuclid", "fp8", 3, 2, 63),
    (133_333, 48, 256, "sqeuclid", "bf16", 1, 0, 64),
    (135_000, 128, 1000, "cosine", "bf16", 3, 1, 65),
    (150_001, 128, 1000, "sqeuclid", "bf16", 2, 1, 66),
    (120_007, 100, 300, "cosine", "bf16", 1, 1, 67),   # two row blocks per wave at depth 128
    (130_001, 128, 1000, "cosine", "bf16", 2, 1, 69),
    (99_999, 120, 129, "sqeuclid", "bf16", 2, 0, 68),
    (131_200, 128, 400, "sqeuclid", "fp8", 2, 2, 70),   # fp8 codes in the GEMM, scaled tables
    (120_001, 72, 300, "cosine", "fp8", 2, 1, 71),
    (60_001, 256, 100, "sqeuclid", "fp8", 2, 0, 72),
]


@pytest.mark.parametrize("case", LARGER_CASES, ids=lambda c: f"N{c[0]}-D{c[1]}-K{c[2]}-{c[3]}-{c[4]}-P{c[5]}")
def test_larger_parity(dev, case):
    n, d, k, metric, form, products, single, seed = case
    b = wl.make_small(n, d, k, seed=seed, singletons=single)
    run_case(dev, b.X, b.labels, k, metric, form, products)


# many clusters: above 16,384 the label histogram leaves LDS for global atomics, above 4,096 the
# scatter places rows one by one, and the sweep runs hundreds of cluster tiles; 65,536 is the limit
@pytest.mark.parametrize("case", [(100_003, 32, 20_000, "sqeuclid", "bf16", 3, 0, 81),
                                  (150_001, 24, 16_385, "cosine", "f32", 0, 1, 82),
                                  (200_000, 8, 65_536, "sqeuclid", "f32", 0, 0, 83)],
                         ids=lambda c: f"N{c[0]}-D{c[1]}-K{c[2]}-{c[3]}-{c[4]}")
def test_many_clusters_parity(dev, case):
    n, d, k, metric, form, products, single, seed = case
    b = wl.make_small(n, d, k, seed=seed, singletons=single)
    run_case(dev, b.X, b.labels, k, metric, form, products)


# approximate Euclidean form (square roots of the point-to-cluster mean squared distances)
APPROX_CASES = [
    # (N, D, K, form, products, singletons, seed)
    (5_037, 40, 70, "f32", 0, 2, 71),
    (3_001, 128, 100, "bf16", 3, 1, 72),
    (4_099, 16, 33, "fp8", 3, 1, 73),
    (140_001, 64, 300, "bf16", 3, 0, 74),
]


@pytest.mark.parametrize("case", APPROX_CASES, ids=lambda c: f"N{c[0]}-D{c[1]}-K{c[2]}-{c[3]}")
def test_euclid_approx_parity(dev, case):
    from paper_2303_14102_amd import binding as sil
    n, d, k, form, products, single, seed = case
    b = wl.make_small(n, d, k, seed=seed, singletons=single)
    Xd, sc, codes = storage(b.X.to(dev), form)
    print(f"[approx] N={n} D={d} K={k} form={form}", flush=True)
    s, S = sil.silhouette(Xd, b.labels.to(dev), k, "sqeuclid", products=products, col_scale=sc,
                          euclid_approx=True, check_status=True)
    cs = None if sc is None else sc.cpu().numpy()
    lab_h = b.labels.numpy()
    s_ref, S_ref, a, bb, _ = oracle.silhouette(codes, lab_h, k, "euclid_approx", col_scale=cs, details=True)
    bound = per_point_bound(form, products, "euclid_approx", True, dequantised(codes, cs), lab_h, k, a, bb)
    s = s.cpu().numpy().astype(np.float64)
    ds = np.abs(s - s_ref)
    print(f"  S={S.item():.10f} ref={S_ref:.10f} max|ds|={ds.max():.2e} max(|ds|/bound)={(ds / bound).max():.3f}",
          flush=True)
    assert np.all(ds <= bound)
    assert abs(S.item() - S_ref) <= TOL_S_MEAN[form]


def test_euclid_approx_argument_errors(dev):
    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(500, 8, 4, seed=75)
    X, lab = b.X.to(dev), b.labels.to(dev)
    for kw in (dict(metric="cosine"), dict(metric="sqeuclid", save_for_grad=True)):
        with pytest.raises(_lib.SilhouetteError) as e:
            sil.silhouette(X, lab, 4, euclid_approx=True, **kw)
        assert e.value.code == -1


def test_uncentred_and_offset_data(dev):
    # far from the origin, centring keeps the bf16 cross term accurate; fp32 too
    b = wl.make_small(4_000, 32, 20, seed=21)
    X = b.X + 1000.0
    for form, products in (("f32", 0), ("bf16", 3)):
        s, S, s_ref, S_ref = run_case(dev, X, b.labels, 20, "sqeuclid", form, products, centre=True)
        assert abs(S - S_ref) <= TOL_S_MEAN[form]
    # folded centring (two products): the cross term's error grows with |x|, within the bound
    run_case(dev, X, b.labels, 20, "sqeuclid", "bf16", 2, centre=True)
    run_case(dev, X, b.labels, 20, "sqeuclid", "fp8", 2, centre=True)
    s, S, s_ref, S_ref = run_case(dev, b.X, b.labels, 20, "sqeuclid", "f32", 0, centre=False)
    assert abs(S - S_ref) <= TOL_S_MEAN["f32"]


def test_two_points(dev):
    # smallest input: two singletons -> s = 0, S = 0
    X = torch.tensor([[0.0, 1.0], [2.0, 3.0]])
    lab = torch.tensor([0, 1], dtype=torch.int32)
    s, S, s_ref, S_ref = run_case(dev, X, lab, 2, "sqeuclid", "f32")
    assert S == 0.0 and np.all(s == 0)


def test_hand_example_on_gpu(dev):
    X = torch.tensor([[0.0], [1.0], [4.0], [6.0]])
    lab = torch.tensor([0, 0, 1, 1], dtype=torch.int32)
    s, S, _, _ = run_case(dev, X, lab, 2, "sqeuclid", "f32")
    want = np.array([25 / 26, 16 / 17, 17 / 25, 53 / 61])
    np.testing.assert_allclose(s, want, atol=1e-6)
    assert abs(S - want.mean()) < 1e-6


# ---------------------------------------------------------------------------------------------
# device-detected errors


def test_device_errors(dev):
    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    X = torch.randn(1000, 8, device=dev)
    lab = torch.randint(0, 4, (1000,), dtype=torch.int32, device=dev)
    ws = sil.new_workspace(1000, 8, 4, "sqeuclid", torch.float32, 0, dev)
    bad = lab.clone()
    bad[17] = 4
    s, S = sil.silhouette(X, bad, 4, workspace=ws)
    assert sil.status(ws) == -3 and math.isnan(S.item()) and torch.isnan(s).all()
    Xn = X.clone()
    Xn[5, 3] = float("nan")
    s, S = sil.silhouette(Xn, lab, 4, workspace=ws)
    assert sil.status(ws) == -6 and math.isnan(S.item())
    one = torch.zeros_like(lab)
    s, S = sil.silhouette(X, one, 4, workspace=ws)
    assert sil.status(ws) == -4 and math.isnan(S.item())
    Xz = X.clone()
    Xz[9] = 0
    wsc = sil.new_workspace(1000, 8, 4, "cosine", torch.float32, 0, dev)
    s, S = sil.silhouette(Xz, lab, 4, "cosine", workspace=wsc)
    assert sil.status(wsc) == -5 and math.isnan(S.item())
    # the same workspace recovers on a good call
    s, S = sil.silhouette(X, lab, 4, workspace=ws)
    assert sil.status(ws) == 0 and not math.isnan(S.item())
    with pytest.raises((ValueError, _lib.SilhouetteError)):
        sil.silhouette(X, lab, 1)


def test_fp8_col_scale_refused_before_launch(dev):
    # a host, strided, wrong-length or float64 col_scale is refused by the binding (a host pointer
    # would reach the kernels otherwise); the output buffers are never touched
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(600, 8, 4, seed=77)
    q, sc = wl.to_fp8_e4m3(b.X.to(dev))
    lab = b.labels.to(dev)
    wide = torch.ones(16, dtype=torch.float32, device=dev)
    for cs in (sc.cpu(), wide[::2], wide[:7], sc.double()):
        with pytest.raises(ValueError):
            sil.silhouette(q, lab, 4, col_scale=cs)
        with pytest.raises(ValueError):
            sil.cluster_stats(q, lab, 4, col_scale=cs)
        with pytest.raises(ValueError):
            sil.silhouette_stream(q.cpu(), b.labels, 4, chunk_rows=256, col_scale=cs, device=dev)
    s, S = sil.silhouette(q, lab, 4, col_scale=sc, check_status=True)
    assert not math.isnan(S.item())


@pytest.mark.parametrize("form,products", [("f32", 0), ("bf16", 2)])
def test_single_call_graph_replay(dev, form, products):
    """One silhouette_sqeuclid call captured into a graph (it launches kernels only) and replayed:
    every replay matches the oracle, with eager library work and a change of X's contents
    between replays (the graph reads X where it lies, so a replay after the change gives the
    Silhouette of the new points)."""
    from paper_2303_14102_amd import binding as sil
    n, d, k = 20_011, 48, 37
    b1 = wl.make_small(n, d, k, seed=91, singletons=2)
    b2 = wl.make_small(n, d, k, seed=92, singletons=1)
    lab = b1.labels.to(dev)
    X1, _, codes1 = storage(b1.X.to(dev), form)
    X2, _, codes2 = storage(b2.X.to(dev), form)
    lab_h = b1.labels.numpy()
    refs = []
    for codes in (codes1, codes2):
        s_ref, S_ref, a, bb, _ = oracle.silhouette(codes, lab_h, k, "sqeuclid", details=True)
        refs.append((s_ref, S_ref, per_point_bound(form, products, "sqeuclid", True,
                                                   dequantised(codes, None), lab_h, k, a, bb)))
    X = X1.clone()
    ws = sil.new_workspace(n, d, k, "sqeuclid", X.dtype, 0, dev)
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        sil.silhouette(X, lab, k, products=products, workspace=ws)  # eager warm-up
    side.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        s_g, S_g = sil.silhouette(X, lab, k, products=products, workspace=ws)
    torch.cuda.current_stream(dev).wait_stream(side)
    ws_other = sil.new_workspace(n, d, k, "cosine", X.dtype, 0, dev)
    for rep, which in enumerate((0, 0, 1, 1, 0)):
        X.copy_(X1 if which == 0 else X2)
        s_g.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert sil.status(ws) == 0
        s_ref, S_ref, bound = refs[which]
        s = s_g.cpu().numpy().astype(np.float64)
        ds = np.abs(s - s_ref)
        print(f"  replay {rep} (X{which + 1}): S={S_g.item():.10f} ref={S_ref:.10f} max|ds|={ds.max():.2e}",
              flush=True)
        assert np.all(ds <= bound), f"replay {rep}: point {int((ds / bound).argmax())}"
        assert abs(S_g.item() - S_ref) <= TOL_S_MEAN[form]
        # eager library work between replays, on another workspace
        sil.silhouette(X2, lab, k, "cosine", products=products, workspace=ws_other, check_status=True)


def test_fp8_every_finite_code(dev):
    """Every finite e4m3fn code (all 256 but the two NaN codes) passes through the library's
    hardware decode: the cluster statistics match the oracle's (which decodes each code by the
    format's definition) to binary64 rounding, and every s_i is within its bound."""
    from paper_2303_14102_amd import binding as sil
    codes_all = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], dtype=np.uint8)
    n, d, k = 2_032, 8, 5  # 254 codes x 8 columns, each code in every column
    rng = np.random.default_rng(131)
    Xc = np.empty((n, d), np.uint8)
    for l in range(d):
        Xc[:, l] = np.tile(np.roll(codes_all, 31 * l), n // len(codes_all))
    labels = rng.integers(0, k, n).astype(np.int32)
    cs = np.ldexp(1.0, rng.integers(-6, 4, d)).astype(np.float32)
    q = torch.from_numpy(Xc).view(torch.float8_e4m3fn).to(dev)
    sc = torch.from_numpy(cs).to(dev)
    lab = torch.from_numpy(labels).to(dev)
    count_g, V_g, psi_g = sil.cluster_stats(q, lab, k, col_scale=sc)
    count, V, psi = oracle.cluster_stats(Xc, labels, k, col_scale=cs)
    assert np.array_equal(count_g.cpu().numpy(), count)
    u = 2.0 ** -53
    tol = 2 * u * count.astype(np.float64)[:, None] ** 2 * np.abs(dequantised(Xc, cs)).max()
    assert np.all(np.abs(V_g.cpu().numpy() - V) <= tol)
    for products in (2, 3):
        s, S = sil.silhouette(q, lab, k, products=products, col_scale=sc, check_status=True)
        s_ref, S_ref, a, bb, _ = oracle.silhouette(Xc, labels, k, col_scale=cs, details=True)
        bound = per_point_bound("fp8", products, "sqeuclid", True, dequantised(Xc, cs), labels, k, a, bb)
        ds = np.abs(s.cpu().numpy().astype(np.float64) - s_ref)
        assert np.all(ds <= bound) and abs(S.item() - S_ref) <= TOL_S_MEAN["fp8"]
