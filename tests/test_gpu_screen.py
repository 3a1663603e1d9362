"""The one-product screen (squared Euclidean, bf16 or fp8 storage, two products): every s_i within
the two-product form's bound of the FP64 oracle and S within 1e-4, next to the plain two-product
sweep (SIL_FLAG_NO_SCREEN) on the same inputs.  Cases cover every screen depth class, K from 2
(one 32-cluster block) to past a thousand, ragged N, singletons and blocks straddling clusters
(excluded per row when clusters are small, deferred to the fallback when N >= 512 K),
and inputs built to send rows to the two-product fallback: exactly tied clusters (duplicated
points), and rows with values beyond fp16's range (values below its finest step are screened with
their rounding in the bound)."""

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


def run_both(dev, X32, labels, K, euclid_approx=False, tag="", form="bf16"):
    """Screen and plain two-product calls on X32 stored bf16 (or fp8 e4m3 with column scales);
    both checked against the oracle."""
    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    Xq, sc, codes = storage(X32.to(dev), form)
    lab = labels.to(dev)
    lab_h = labels.numpy()
    cs = None if sc is None else sc.cpu().numpy()
    metric = "euclid_approx" if euclid_approx else "sqeuclid"
    s_ref, S_ref, a, bb, _ = oracle.silhouette(codes, lab_h, K, metric, col_scale=cs, details=True)
    bound = per_point_bound(form, 2, metric, True, dequantised(codes, cs), lab_h, K, a, bb)
    n, d = Xq.shape
    out = {}
    for screen in (True, False):
        flags = (_lib.SIL_FLAG_EUCLID_APPROX if euclid_approx else 0) | (0 if screen else _lib.SIL_FLAG_NO_SCREEN)
        ws = sil.new_workspace(n, d, K, "sqeuclid", Xq.dtype, flags, dev)
        s = torch.full((n,), float("nan"), dtype=torch.float32, device=dev)
        S = torch.empty((), dtype=torch.float64, device=dev)
        rc = _lib.load().silhouette_sqeuclid(sil._ptr(Xq), sil._dtype_code(Xq), sil._ptr(sc), sil._ptr(lab), n, d,
                                             K, 2, flags, sil._ptr(s), sil._ptr(S), sil._ptr(ws), ws.numel(),
                                             sil._stream(dev))
        _lib.check(rc, "silhouette_sqeuclid")
        torch.cuda.synchronize()
        assert sil.status(ws) == 0
        fb = sil.fallback_rows(ws) if screen else None
        sv = s.cpu().numpy().astype(np.float64)
        ds = np.abs(sv - s_ref)
        print(f"  {tag} screen={screen}: S={S.item():.12f} ref={S_ref:.12f} |dS|={abs(S.item() - S_ref):.2e} "
              f"max|ds|={ds.max():.2e} max(|ds|/bound)={(ds / bound).max():.4f} fallback={fb}", flush=True)
        assert np.all(ds <= bound), f"{tag} screen={screen}: point {int((ds / bound).argmax())}"
        assert abs(S.item() - S_ref) <= TOL_S_MEAN[form]
        out[screen] = (sv, S.item(), fb)
    return out


# (N, D, K, singletons, seed)
CASES = [
    (3_001, 16, 2, 0, 101),      # one 32-cluster block, one tile
    (5_003, 16, 33, 1, 102),
    (9_999, 32, 64, 2, 103),
    (20_011, 48, 100, 0, 104),
    (30_007, 64, 250, 3, 105),
    (12_345, 96, 97, 1, 106),
    (40_009, 128, 1000, 2, 107),
    (7_777, 128, 2050, 0, 108),  # more clusters than rows in some blocks; K past 2048
    (255, 128, 7, 1, 109),       # fewer rows than one workgroup
    # N >= 512 K: blocks that straddle a cluster boundary go whole to the fallback
    (60_013, 128, 100, 1, 131),  # D equal to the depth class
    (40_009, 100, 64, 2, 132),   # D below it
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c[0]}-D{c[1]}-K{c[2]}")
def test_screen_parity(dev, case):
    n, d, k, single, seed = case
    print(f"[screen] N={n} D={d} K={k} singletons={single}", flush=True)
    b = wl.make_small(n, d, k, seed=seed, singletons=single)
    out = run_both(dev, b.X, b.labels, k, tag=f"N{n}-D{d}-K{k}")
    assert out[True][2] <= n


def test_screen_tied_clusters_go_to_the_fallback(dev):
    # cluster 7 is an exact copy of cluster 3's points: the two have the same mean and spread, so
    # every row whose nearest other cluster is one of them sees an exact tie
    n, d, k = 20_000, 64, 40
    b = wl.make_small(n, d, k, seed=111)
    X, lab = b.X.clone(), b.labels.clone()
    src = torch.nonzero(lab == 3).flatten()
    dst = torch.nonzero(lab == 7).flatten()
    m = min(len(src), len(dst))
    keep = torch.ones(n, dtype=torch.bool)
    keep[dst[m:]] = False  # drop the extra rows of cluster 7 so that the two clusters match exactly
    X[dst[:m]] = X[src[:m]]
    X, lab = X[keep], lab[keep]
    print(f"[screen] tied clusters: N={len(lab)} copies={m}", flush=True)
    out = run_both(dev, X, lab, k, tag="tied")
    assert out[True][2] > 0


def test_screen_rows_outside_fp16(dev):
    # a row beyond fp16's range goes to the fallback; rows with values below fp16's finest step
    # are screened (their rounding, under 2^-24 a value, is in the bound)
    n, d, k = 15_000, 32, 25
    b = wl.make_small(n, d, k, seed=112)
    X = b.X.clone()
    X[5] *= 1.0e5
    X[77, :4] = 3.0e-8
    X[1234, 3] = -7.5e-9
    print("[screen] rows outside fp16", flush=True)
    out = run_both(dev, X, b.labels, k, tag="fp16-range")
    assert out[True][2] >= 1


def test_screen_tiny_values(dev):
    # data scaled far down (many values below fp16's normal range): rows too small for the exact
    # score from fp16 values go to the fallback; moderately small data is screened
    b = wl.make_small(12_000, 64, 30, seed=115)
    print("[screen] tiny values", flush=True)
    out = run_both(dev, b.X * 1.0e-5, b.labels, 30, tag="tiny")
    assert out[True][2] > 11_000
    out = run_both(dev, b.X * 1.0e-2, b.labels, 30, tag="small")
    assert out[True][2] < 2_000


def test_screen_euclid_approx(dev):
    b = wl.make_small(25_000, 64, 150, seed=113, singletons=1)
    print("[screen] approximate Euclidean form", flush=True)
    run_both(dev, b.X, b.labels, 150, euclid_approx=True, tag="approx")


def test_screen_offset_data(dev):
    # far from the origin: the folded centring's cross term and the screen's bound grow with |x|;
    # more rows fall back, and the results stay within the two-product bound
    b = wl.make_small(20_000, 32, 60, seed=114)
    print("[screen] offset data", flush=True)
    out = run_both(dev, b.X + 300.0, b.labels, 60, tag="offset")
    print(f"  fallback rows: {out[True][2]}", flush=True)


FP8_CASES = [
    (9_999, 16, 40, 1, 121),
    (20_011, 64, 100, 0, 122),
    (30_007, 96, 257, 2, 123),
    (40_009, 128, 1000, 1, 124),
    (50_021, 128, 80, 1, 133),   # N >= 512 K: straddling blocks go to the fallback
]


@pytest.mark.parametrize("case", FP8_CASES, ids=lambda c: f"N{c[0]}-D{c[1]}-K{c[2]}")
def test_screen_fp8_parity(dev, case):
    # fp8 e4m3 storage: the codes enter the screen (exact in fp16), the table carries the scales
    n, d, k, single, seed = case
    print(f"[screen fp8] N={n} D={d} K={k}", flush=True)
    b = wl.make_small(n, d, k, seed=seed, singletons=single)
    out = run_both(dev, b.X, b.labels, k, tag=f"fp8-N{n}-D{d}-K{k}", form="fp8")
    assert out[True][2] < n // 4


def test_screen_fp8_unscreened_shapes(dev):
    # D not a multiple of 8: the fp8 call runs the two-product sweep (no rows are listed)
    b = wl.make_small(8_000, 20, 30, seed=125)
    out = run_both(dev, b.X, b.labels, 30, tag="fp8-D20", form="fp8")
    assert out[True][2] == 0
