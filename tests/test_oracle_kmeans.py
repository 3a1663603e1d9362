"""Pins of the oracle's K-means (Lloyd) step, CPU only:
- hand-worked steps with closed-form labels and inertia (tests/golden/kmeans_examples.json);
- scipy.cluster.vq.vq (a library routine for nearest-centroid assignment) against the oracle's
  assignment, with the means taken by numpy from the labels;
- Lloyd's monotonicity: the new inertia is at most the old labels' distance to the same means;
- a fixed point on well-separated blobs, empty ids staying empty, the error conventions.
"""

import json
import os

import numpy as np
import pytest
from scipy.cluster.vq import vq

import oracle
from paper_2303_14102_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "kmeans_examples.json")


@pytest.mark.parametrize("ex", json.load(open(GOLDEN))["examples"], ids=lambda e: e["name"])
def test_kmeans_hand_examples(ex):
    X = np.array(ex["X"], dtype=np.float64)
    lab, inertia, d1, d2 = oracle.kmeans_step(X, np.array(ex["labels"]), ex["K"])
    assert lab.tolist() == ex["labels_out"]
    assert inertia == float(ex["inertia"])
    assert abs(d1.sum() - inertia) == 0.0


def numpy_means(X, labels, K):
    ids = np.unique(labels)
    return ids, np.stack([X[labels == k].mean(axis=0) for k in ids])


@pytest.mark.parametrize("n,d,k,unused,seed", [(3_000, 5, 7, 2, 1), (5_000, 32, 40, 5, 2), (1_000, 128, 3, 0, 3)])
def test_kmeans_matches_scipy_vq(n, d, k, unused, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d)) * 2.0
    labels = rng.integers(0, k, size=n).astype(np.int32)
    labels[labels < unused] = unused  # ids below `unused` are empty
    lab, inertia, d1, d2 = oracle.kmeans_step(X, labels, k)
    ids, means = numpy_means(X, labels, k)
    code, dist = vq(X, means)
    np.testing.assert_array_equal(lab, ids[code])
    np.testing.assert_allclose(d1, dist ** 2, rtol=1e-12, atol=1e-12)
    assert abs(inertia - (dist ** 2).sum()) <= 1e-10 * inertia
    assert np.all(d2 >= d1)
    assert not np.isin(lab, np.arange(unused)).any()


def test_kmeans_inertia_does_not_increase():
    b = wl.make_small(4_000, 16, 12, seed=5, sigma=4.0, relabel=0.3)
    X, labels = b.X.numpy().astype(np.float64), b.labels.numpy()
    lab, inertia, _, _ = oracle.kmeans_step(X, labels, 12)
    ids, means = numpy_means(X, labels, 12)
    pos = {int(k): i for i, k in enumerate(ids)}
    old = sum(((X[labels == k] - means[pos[int(k)]]) ** 2).sum() for k in ids)
    assert inertia <= old
    assert (lab != labels).sum() > 0  # the noisy labels do move
    # a second step from the new labels again does not increase it
    _, inertia2, _, _ = oracle.kmeans_step(X, lab, 12)
    assert inertia2 <= inertia * (1 + 1e-15)


def test_kmeans_fixed_point_on_separated_blobs():
    b = wl.make_small(6_000, 16, 8, seed=6, sigma=0.3, relabel=0.0)
    lab, _, d1, d2 = oracle.kmeans_step(b.X.numpy(), b.labels.numpy(), 8)
    np.testing.assert_array_equal(lab, b.labels.numpy())
    assert np.all(d2 > d1)


def test_kmeans_storage_forms_decode_like_the_silhouette():
    # bf16 bit patterns and fp8 codes with a column scale give the step on the decoded values
    import torch
    b = wl.make_small(2_000, 24, 6, seed=7)
    for form in ("bf16", "fp8"):
        if form == "bf16":
            codes = b.X.to(torch.bfloat16).view(torch.uint16).numpy()
            dec, cs = b.X.to(torch.bfloat16).float().numpy().astype(np.float64), None
        else:
            q, scale = wl.to_fp8_e4m3(b.X)
            codes, cs = q.view(torch.uint8).numpy(), scale.numpy()
            dec = q.float().numpy().astype(np.float64) * scale.numpy().astype(np.float64)
        got = oracle.kmeans_step(codes, b.labels.numpy(), 6, col_scale=cs)
        want = oracle.kmeans_step(dec, b.labels.numpy(), 6)
        np.testing.assert_array_equal(got[0], want[0])
        assert got[1] == want[1]


def test_kmeans_errors():
    X = np.zeros((4, 2))
    with pytest.raises(oracle.OracleError) as e:
        oracle.kmeans_step(X, np.array([0, 1, 2, 0]), 2)
    assert e.value.code == -3
    X[1, 1] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.kmeans_step(X, np.array([0, 1, 1, 0]), 2)
    assert e.value.code == -6
