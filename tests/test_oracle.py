"""Pins for the FP64 oracle, each against something other than the oracle itself.

- hand-worked examples with closed-form answers (tests/golden/hand_examples.json);
- the quadratic definition written out here in numpy, and scikit-learn's silhouette_samples
  (a library routine for Eq.1 with the singleton convention);
- invariants of the definition (range, permutation, renaming, unused ids, translation,
  rotation and scale for squared Euclidean, per-row positive scaling for cosine, duplicate-point
  clusters, partition of the statistics);
- the storage decoders against torch's own bf16 / fp8 e4m3fn conversions;
- the derived gradient against torch float64 autograd through the quadratic definition, and
  central finite differences of the oracle's S;
- the error conventions.
"""

import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2303_14102_amd import workloads as wl

SK_METRIC = {"sqeuclid": "sqeuclidean", "cosine": "cosine"}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _eval_closed_form(expr: str) -> float:
    return float(eval(expr, {"__builtins__": {}}, {"sqrt": math.sqrt, "log": math.log}))


# ---------------------------------------------------------------------------------------------
# hand-worked examples


@pytest.mark.parametrize("ex", json.load(open(GOLDEN))["examples"], ids=lambda e: e["name"])
def test_hand_examples(ex):
    X = np.array(ex["X"], dtype=np.float64)
    labels = np.array(ex["labels"], dtype=np.int32)
    want = np.array([_eval_closed_form(e) for e in ex["s"]])
    s, S = oracle.silhouette(X, labels, ex["K"], ex["metric"])
    np.testing.assert_allclose(s, want, rtol=0, atol=1e-14)
    assert abs(S - want.mean()) < 1e-14
    sb, Sb = oracle.brute_silhouette(X, labels, ex["K"], ex["metric"])
    np.testing.assert_allclose(sb, want, rtol=0, atol=1e-14)


def test_hand_example_e1_exact_mean():
    # S for E1 as one exact fraction: (25/26 + 16/17 + 17/25 + 53/61) / 4
    from fractions import Fraction as F
    want = (F(25, 26) + F(16, 17) + F(17, 25) + F(53, 61)) / 4
    assert want == F(2326529, 2696200)
    _, S = oracle.silhouette(np.array([[0.], [1.], [4.], [6.]]), np.array([0, 0, 1, 1], np.int32), 2)
    assert abs(S - float(want)) < 1e-15


# ---------------------------------------------------------------------------------------------
# the quadratic definition, written independently here


def numpy_brute(X, labels, K, metric):
    X = np.asarray(X, np.float64)
    if metric == "sqeuclid":
        # pairwise differences, not the expansion the oracle uses
        Dm = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    else:
        Z = X / np.linalg.norm(X, axis=1, keepdims=True)
        Dm = 1.0 - Z @ Z.T
        np.fill_diagonal(Dm, 0.0)
    N = len(X)
    cnt = np.bincount(labels, minlength=K)
    s = np.zeros(N)
    for i in range(N):
        o = labels[i]
        if cnt[o] < 2:
            continue
        sums = np.bincount(labels, weights=Dm[i], minlength=K)
        a = sums[o] / (cnt[o] - 1)
        others = [sums[k] / cnt[k] for k in range(K) if k != o and cnt[k] > 0]
        b = min(others)
        mx = max(a, b)
        s[i] = 0.0 if mx == 0 else (b - a) / mx
    return s, s.mean()


def _random_case(rng, n, d, k, singletons=1, unused=1):
    X = rng.normal(size=(n, d)) * rng.uniform(0.5, 2.0) + rng.integers(-3, 4, size=d)
    labels = rng.integers(0, k, size=n).astype(np.int32)
    # make the first `singletons` ids singletons and leave `unused` ids empty
    K = k + singletons + unused
    for t in range(singletons):
        labels[t] = k + t
    return X, labels, K


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_oracle_matches_quadratic_definition(metric, seed):
    rng = np.random.default_rng(100 + seed)
    X, labels, K = _random_case(rng, n=60 + 17 * seed, d=2 + seed, k=3 + seed)
    s, S = oracle.silhouette(X, labels, K, metric)
    s_ref, S_ref = numpy_brute(X, labels, K, metric)
    np.testing.assert_allclose(s, s_ref, rtol=0, atol=1e-12)
    assert abs(S - S_ref) < 1e-12
    s_b, S_b = oracle.brute_silhouette(X, labels, K, metric)
    np.testing.assert_allclose(s_b, s_ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_oracle_matches_sklearn(metric, seed):
    sk = pytest.importorskip("sklearn.metrics")
    rng = np.random.default_rng(200 + seed)
    X, labels, K = _random_case(rng, n=300 + 100 * seed, d=3 + 2 * seed, k=4 + seed, unused=0)
    s, S = oracle.silhouette(X, labels, K, metric)
    s_ref = sk.silhouette_samples(X, labels, metric=SK_METRIC[metric])
    np.testing.assert_allclose(s, s_ref, rtol=0, atol=1e-10)
    assert abs(S - s_ref.mean()) < 1e-12


def test_oracle_matches_sklearn_on_blobs():
    sk = pytest.importorskip("sklearn.metrics")
    b = wl.make_small(2000, 8, 6, seed=5, singletons=1)
    X = b.X.numpy()
    lab = b.labels.numpy()
    for metric in ("sqeuclid", "cosine"):
        s, S = oracle.silhouette(X, lab, 6, metric)
        s_ref = sk.silhouette_samples(X.astype(np.float64), lab, metric=SK_METRIC[metric])
        np.testing.assert_allclose(s, s_ref, rtol=0, atol=1e-9)


# ---------------------------------------------------------------------------------------------
# invariants


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(7)
    X, labels, K = _random_case(rng, n=400, d=5, k=5)
    return X, labels, K


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
def test_range_permutation_renaming(case, metric):
    X, labels, K = case
    s, S = oracle.silhouette(X, labels, K, metric)
    assert np.all(s >= -1 - 1e-15) and np.all(s <= 1 + 1e-15) and -1 <= S <= 1
    perm = np.random.default_rng(1).permutation(len(X))
    s2, S2 = oracle.silhouette(X[perm], labels[perm], K, metric)
    np.testing.assert_allclose(s2, s[perm], atol=1e-12)
    assert abs(S2 - S) < 1e-13
    ren = np.random.default_rng(2).permutation(K + 3).astype(np.int32)  # also adds unused ids
    s3, S3 = oracle.silhouette(X, ren[labels], K + 3, metric)
    np.testing.assert_allclose(s3, s, atol=1e-12)


def test_sqeuclid_rigid_and_scale_invariance(case):
    X, labels, K = case
    s, S = oracle.silhouette(X, labels, K, "sqeuclid")
    Q, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(X.shape[1],) * 2))
    Y = 3.5 * (X @ Q) + np.arange(X.shape[1]) * 7.0
    s2, S2 = oracle.silhouette(Y, labels, K, "sqeuclid")
    np.testing.assert_allclose(s2, s, atol=1e-10)


def test_cosine_row_scale_invariance(case):
    X, labels, K = case
    s, _ = oracle.silhouette(X, labels, K, "cosine")
    scale = np.random.default_rng(4).uniform(0.01, 100.0, size=(len(X), 1))
    s2, _ = oracle.silhouette(X * scale, labels, K, "cosine")
    np.testing.assert_allclose(s2, s, atol=1e-12)


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
def test_duplicate_point_clusters(metric):
    # every cluster is copies of one point (for cosine: positive multiples of one direction):
    # a_i = 0 and b_i > 0, so s_i = 1, except singletons (0): S = (points in clusters of size >= 2)/N
    rng = np.random.default_rng(9)
    K, D = 6, 4
    base = rng.normal(size=(K, D))
    sizes = np.array([5, 1, 7, 3, 1, 9])
    labels = np.repeat(np.arange(K), sizes).astype(np.int32)
    X = base[labels].copy()
    if metric == "cosine":
        X *= rng.uniform(0.5, 2.0, size=(len(X), 1))
    s, S = oracle.silhouette(X, labels, K, metric)
    want = np.where(sizes[labels] >= 2, 1.0, 0.0)
    np.testing.assert_allclose(s, want, atol=1e-12)
    assert abs(S - (sizes[sizes >= 2].sum() / sizes.sum())) < 1e-12


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
def test_stats_partition_invariance(case, metric):
    # per-shard statistics summed equal the statistics of the whole (footnote to Eq.6)
    X, labels, K = case
    c, V, p = oracle.cluster_stats(X, labels, K, metric)
    acc = [np.zeros_like(c), np.zeros_like(V), np.zeros_like(p)]
    for part in np.array_split(np.arange(len(X)), 4):
        cs, Vs, ps = oracle.cluster_stats(X[part], labels[part], K, metric)
        acc[0] += cs
        acc[1] += Vs
        acc[2] += ps
    assert np.array_equal(acc[0], c)
    np.testing.assert_allclose(acc[1], V, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(acc[2], p, rtol=1e-13)
    # and the statistics themselves by their definitions
    assert np.array_equal(c, np.bincount(labels, minlength=K))
    if metric == "sqeuclid":
        for k in range(K):
            np.testing.assert_allclose(V[k], X[labels == k].sum(0), rtol=1e-13, atol=1e-12)
            np.testing.assert_allclose(p[k], (X[labels == k] ** 2).sum(), rtol=1e-13)


def test_scores_at_matches_full(case):
    X, labels, K = case
    s, S = oracle.silhouette(X, labels, K)
    st = oracle.cluster_stats(X, labels, K)
    idx = np.array([0, 5, 17, 399, 5])
    s2, a, b, nbr = oracle.scores_at(X, labels, K, idx, st)
    np.testing.assert_array_equal(s2, s[idx])


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
def test_brute_scores_at_matches_sklearn(metric):
    # the per-point quadratic definition (used on sampled points of large workloads) against the
    # library routine on the same points, including a singleton cluster
    sk = pytest.importorskip("sklearn.metrics")
    b = wl.make_small(700, 6, 9, seed=5, singletons=1)
    X, lab = b.X.numpy().astype(np.float64), b.labels.numpy()
    idx = np.array([0, 3, 77, 350, 699, 3])
    s, a, bb = oracle.brute_scores_at(X, lab, 9, idx, metric)
    ref = sk.silhouette_samples(X, lab, metric=SK_METRIC[metric])
    np.testing.assert_allclose(s, ref[idx], rtol=1e-12, atol=1e-13)
    s_full, _ = oracle.brute_silhouette(X, lab, 9, metric)
    np.testing.assert_allclose(s, s_full[idx], rtol=1e-12, atol=1e-13)
    s_lin, a_lin, b_lin, _ = oracle.scores_at(X, lab, 9, idx, oracle.cluster_stats(X, lab, 9, metric), metric)
    np.testing.assert_allclose(a, a_lin, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(s, s_lin, rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------------------------------------
# approximate Euclidean form (Section V): square roots of the point-to-cluster mean squared
# distances


def test_euclid_approx_equals_exact_where_distances_to_a_cluster_are_equal():
    # cluster j = {r_j e_j, -r_j e_j} on its own axis: every distance from a point to the members
    # of a cluster is the same, so the root of the mean squared distance is the mean distance and
    # the approximation equals the exact Euclidean Silhouette (scikit-learn); plus a singleton
    sk = pytest.importorskip("sklearn.metrics")
    rng = np.random.default_rng(17)
    K = 6
    r = rng.uniform(0.5, 4.0, size=K)
    X = np.zeros((2 * K + 1, K + 1))
    lab = np.zeros(2 * K + 1, np.int32)
    for j in range(K):
        X[2 * j, j], X[2 * j + 1, j] = r[j], -r[j]
        lab[2 * j] = lab[2 * j + 1] = j
    X[2 * K, K] = 2.5          # alone in cluster K
    lab[2 * K] = K
    s, S = oracle.silhouette(X, lab, K + 1, "euclid_approx")
    ref = sk.silhouette_samples(X, lab, metric="euclidean")
    np.testing.assert_allclose(s, ref, rtol=0, atol=1e-13)
    assert s[-1] == 0.0 and len(set(np.round(s[:-1], 6))) > 3  # non-trivial values


@pytest.mark.parametrize("seed", [0, 1])
def test_euclid_approx_definition_and_jensen(seed):
    # the linear form equals the quadratic definition of the approximation, and each root of a
    # mean squared distance is at least the mean Euclidean distance (Jensen), so a' >= a, b' >= b
    rng = np.random.default_rng(300 + seed)
    X, labels, K = _random_case(rng, n=250, d=5, k=6, unused=1)
    s, S, a, b, _ = oracle.silhouette(X, labels, K, "euclid_approx", details=True)
    sb, Sb = oracle.brute_silhouette(X, labels, K, "euclid_approx")
    np.testing.assert_allclose(s, sb, rtol=0, atol=1e-10)
    dist = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))
    cnt = np.bincount(labels, minlength=K)
    for i in range(len(X)):
        o = labels[i]
        if cnt[o] < 2:
            continue
        a_exact = dist[i, labels == o].sum() / (cnt[o] - 1)
        b_exact = min(dist[i, labels == k].mean() for k in range(K) if k != o and cnt[k] > 0)
        assert a[i] >= a_exact - 1e-12 and b[i] >= b_exact - 1e-12
    s2, a2, b2 = oracle.brute_scores_at(X, labels, K, np.arange(len(X)), "euclid_approx")
    np.testing.assert_allclose(s2, sb, rtol=0, atol=1e-13)
    with pytest.raises(oracle.OracleError):
        oracle.gradient(X, labels, K, "euclid_approx")


def test_expanded_form_vs_centred_form_at_offset():
    # Eq.11 expanded versus the centred form ||x - mu_k||^2 + sigma_k^2 (exact algebra),
    # evaluated in binary64 on data far from the origin
    b = wl.make_small(3000, 16, 8, seed=11)
    X = b.X.numpy().astype(np.float64) + 50.0
    lab = b.labels.numpy()
    s, S, a, bb, nbr = oracle.silhouette(X, lab, 8, details=True)
    cnt = np.bincount(lab, minlength=8)
    mu = np.stack([X[lab == k].mean(0) for k in range(8)])
    var = np.array([((X[lab == k] - mu[k]) ** 2).sum(1).mean() for k in range(8)])
    m = ((X[:, None, :] - mu[None]) ** 2).sum(-1) + var[None]
    a2 = m[np.arange(len(X)), lab] * cnt[lab] / (cnt[lab] - 1)
    m[np.arange(len(X)), lab] = np.inf
    np.testing.assert_allclose(a, a2, rtol=1e-10)
    np.testing.assert_allclose(bb, m.min(1), rtol=1e-10)


# ---------------------------------------------------------------------------------------------
# storage decoders


def test_decode_bf16_matches_torch():
    bits = np.concatenate([np.arange(0, 65536, 37, dtype=np.uint16), np.array([0x3F80, 0xBF80, 0x0001, 0x7F7F], np.uint16)])
    ref = torch.from_numpy(bits.view(np.int16)).view(torch.bfloat16).float().numpy().astype(np.float64)
    got = np.array([oracle.decode_bf16(int(h)) for h in bits])
    finite = np.isfinite(ref)
    np.testing.assert_array_equal(got[finite], ref[finite])
    assert np.all(np.isnan(got[np.isnan(ref)]))


def test_decode_e4m3_matches_torch():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    got = np.array([oracle.decode_e4m3(int(q)) for q in codes])
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    np.testing.assert_array_equal(got[~nan], ref[~nan])


def test_quantised_inputs_use_exact_dequantisation():
    b = wl.make_small(500, 8, 4, seed=3)
    q16 = wl.to_bf16(b.X)
    codes = wl.host_codes(q16)
    deq = q16.float().numpy()
    lab = b.labels.numpy()
    s1, S1 = oracle.silhouette(codes, lab, 4)
    s2, S2 = oracle.silhouette(deq, lab, 4)
    np.testing.assert_array_equal(s1, s2)
    q8, scale = wl.to_fp8_e4m3(b.X)
    deq8 = (q8.float() * scale).numpy()
    s3, _ = oracle.silhouette(wl.host_codes(q8), lab, 4, col_scale=scale.numpy())
    s4, _ = oracle.silhouette(deq8, lab, 4)
    np.testing.assert_array_equal(s3, s4)


# ---------------------------------------------------------------------------------------------
# gradient


def torch_brute_S(X, labels, K, metric):
    N = X.shape[0]
    if metric == "sqeuclid":
        Dm = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    else:
        Z = X / X.norm(dim=1, keepdim=True)
        Dm = 1.0 - Z @ Z.T
        Dm = Dm - torch.diag(torch.diag(Dm))
    lab = torch.as_tensor(labels, dtype=torch.long)
    onehot = torch.nn.functional.one_hot(lab, K).to(X.dtype)
    cnt = onehot.sum(0)
    sums = Dm @ onehot  # [N, K]
    s = []
    for i in range(N):
        o = int(lab[i])
        if cnt[o] < 2:
            s.append(torch.zeros((), dtype=X.dtype))
            continue
        a = sums[i, o] / (cnt[o] - 1)
        others = torch.stack([sums[i, k] / cnt[k] for k in range(K) if k != o and cnt[k] > 0])
        b = others.min()
        s.append((b - a) / torch.maximum(a, b))
    return torch.stack(s).sum() / N


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_autograd_of_definition(metric, seed):
    rng = np.random.default_rng(300 + seed)
    X, labels, K = _random_case(rng, n=23 + seed * 9, d=3, k=3)
    Xt = torch.tensor(X, dtype=torch.float64, requires_grad=True)
    S = torch_brute_S(Xt, labels, K, metric)
    S.backward()
    g = oracle.gradient(X, labels, K, metric)
    np.testing.assert_allclose(g, Xt.grad.numpy(), rtol=0, atol=1e-13)
    _, S_or = oracle.silhouette(X, labels, K, metric)
    assert abs(S_or - S.item()) < 1e-13


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
def test_gradient_matches_finite_differences(metric):
    b = wl.make_small(800, 6, 5, seed=21, sigma=1.5)
    X = b.X.numpy().astype(np.float64)
    lab = b.labels.numpy()
    g = oracle.gradient(X, lab, 5, metric)
    rng = np.random.default_rng(5)
    h = 1e-5
    for _ in range(12):
        i, l = int(rng.integers(len(X))), int(rng.integers(X.shape[1]))
        Xp, Xm = X.copy(), X.copy()
        Xp[i, l] += h
        Xm[i, l] -= h
        fd = (oracle.silhouette(Xp, lab, 5, metric)[1] - oracle.silhouette(Xm, lab, 5, metric)[1]) / (2 * h)
        assert abs(fd - g[i, l]) <= 1e-7 * max(1.0, abs(g[i, l])) + 1e-9, (i, l, fd, g[i, l])


# ---------------------------------------------------------------------------------------------
# error conventions


def test_errors():
    X = np.zeros((4, 2))
    X[:, 0] = [1, 2, 3, 4]
    with pytest.raises(oracle.OracleError) as e:
        oracle.silhouette(X, np.array([0, 1, 2, 0], np.int32), 2)
    assert e.value.code == -3
    with pytest.raises(oracle.OracleError) as e:
        oracle.silhouette(X, np.array([0, 0, 0, 0], np.int32), 2)
    assert e.value.code == -4
    Xn = X.copy()
    Xn[2, 1] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.silhouette(Xn, np.array([0, 1, 0, 1], np.int32), 2)
    assert e.value.code == -6
    Xz = X.copy()
    Xz[1] = 0
    with pytest.raises(oracle.OracleError) as e:
        oracle.silhouette(Xz, np.array([0, 1, 0, 1], np.int32), 2, "cosine")
    assert e.value.code == -5
    # the zero row is fine under the squared Euclidean distance
    oracle.silhouette(Xz, np.array([0, 1, 0, 1], np.int32), 2, "sqeuclid")


def test_all_points_singletons_or_two_clusters_minimum():
    X = np.array([[0.0], [1.0]])
    s, S = oracle.silhouette(X, np.array([0, 1], np.int32), 2)
    assert S == 0.0 and np.all(s == 0)
