"""Pins of the oracle's generalized Kullback-Leibler Silhouette (the Bregman divergence of
phi(x) = sum x log x - x, point first), CPU only; the hand-worked example E5 sits with the others in
tests/golden/hand_examples.json:
- the linear form against its own quadratic definition and against scikit-learn's
  silhouette_samples on a divergence matrix built here in numpy (metric="precomputed");
- invariance to scaling all data (the divergence is 1-homogeneous); identical points give s = 1;
- the domain error for non-positive entries, and no gradient.
"""

import numpy as np
import pytest
from sklearn.metrics import silhouette_samples

import oracle


def positive_case(seed, n=90, d=6, k=4):
    rng = np.random.default_rng(seed)
    labels = rng.integers(0, k, size=n).astype(np.int32)
    centres = rng.normal(0.0, 1.0, size=(k, d))
    X = np.exp(centres[labels] + 0.4 * rng.standard_normal((n, d)))
    return X, labels


def kl_matrix(X):
    return (X[:, None, :] * np.log(X[:, None, :] / X[None, :, :]) - X[:, None, :] + X[None, :, :]).sum(-1)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_linear_equals_quadratic_and_sklearn(seed):
    X, labels = positive_case(seed)
    s, S = oracle.silhouette(X, labels, 4, "kl")
    sb, Sb = oracle.brute_silhouette(X, labels, 4, "kl")
    np.testing.assert_allclose(s, sb, rtol=0, atol=1e-12)
    Dm = kl_matrix(X)
    np.fill_diagonal(Dm, 0.0)
    np.testing.assert_allclose(s, silhouette_samples(Dm, labels, metric="precomputed"), rtol=0, atol=1e-12)
    assert abs(S - s.mean()) < 1e-15
    # the sampled quadratic form agrees too
    idx = np.array([0, 5, 17, 89])
    sa, _, _ = oracle.brute_scores_at(X, labels, 4, idx, "kl")
    np.testing.assert_allclose(sa, s[idx], rtol=0, atol=1e-12)


def test_scale_invariance_and_identical_points():
    X, labels = positive_case(3)
    s, _ = oracle.silhouette(X, labels, 4, "kl")
    s2, _ = oracle.silhouette(7.25 * X, labels, 4, "kl")
    np.testing.assert_allclose(s, s2, rtol=0, atol=1e-12)
    Y = np.repeat(np.array([[1.0, 2.0], [5.0, 0.5], [3.0, 3.0]]), 4, axis=0)
    s3, S3 = oracle.silhouette(Y, np.repeat(np.arange(3, dtype=np.int32), 4), 3, "kl")
    np.testing.assert_allclose(s3, 1.0, rtol=0, atol=1e-12)


def test_domain_and_gradient_errors():
    X, labels = positive_case(4, n=12)
    X[3, 2] = 0.0
    for fn in (oracle.silhouette, oracle.brute_silhouette):
        with pytest.raises(oracle.OracleError) as e:
            fn(X, labels, 4, "kl")
        assert e.value.code == -10
    X[3, 2] = 1.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.gradient(X, labels, 4, "kl")
    assert e.value.code == -1
