"""Pins of the oracle's fixed-matrix Mahalanobis Silhouette, d(x, y) = (x - y)^T M (x - y), CPU only:
- the linear form against its own quadratic definition and against scikit-learn's
  silhouette_samples on a distance matrix built here in numpy (metric="precomputed");
- M = I is the squared Euclidean Silhouette; a diagonal M is the squared Euclidean one on scaled
  columns; s is unchanged when M is scaled, and under a change of basis x -> A x with
  M -> A^-T M A^-1; a rank-deficient M; the error conventions.
"""

import numpy as np
import pytest
from sklearn.metrics import silhouette_samples

import oracle


def random_case(seed, n=80, d=6, k=4, rank=None):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d)) + rng.integers(-3, 4, size=(1, d))
    labels = rng.integers(0, k, size=n).astype(np.int32)
    L = rng.standard_normal((rank or d, d))
    return X, labels, L.T @ L


def pairwise(X, M):
    diff = X[:, None, :] - X[None, :, :]
    return np.einsum("ijl,lm,ijm->ij", diff, M, diff)


@pytest.mark.parametrize("seed,rank", [(0, None), (1, None), (2, 3), (3, 1)])
def test_linear_equals_quadratic_and_sklearn(seed, rank):
    X, labels, M = random_case(seed, rank=rank)
    s, S = oracle.silhouette_mahalanobis(X, labels, 4, M)
    sb, Sb = oracle.brute_silhouette_mahalanobis(X, labels, 4, M)
    np.testing.assert_allclose(s, sb, rtol=0, atol=1e-12)
    D2 = pairwise(X, M)
    np.fill_diagonal(D2, 0.0)
    np.testing.assert_allclose(s, silhouette_samples(D2, labels, metric="precomputed"), rtol=0, atol=1e-12)
    assert abs(S - s.mean()) < 1e-15


def test_identity_is_squared_euclidean():
    X, labels, _ = random_case(4)
    s, _ = oracle.silhouette_mahalanobis(X, labels, 4, np.eye(X.shape[1]))
    s_e, _ = oracle.silhouette(X, labels, 4, "sqeuclid")
    np.testing.assert_allclose(s, s_e, rtol=0, atol=1e-13)


def test_diagonal_is_scaled_columns():
    X, labels, _ = random_case(5)
    w = np.array([0.5, 2.0, 1.0, 3.0, 0.25, 1.5])
    s, _ = oracle.silhouette_mahalanobis(X, labels, 4, np.diag(w ** 2))
    s_e, _ = oracle.silhouette(X * w, labels, 4, "sqeuclid")
    np.testing.assert_allclose(s, s_e, rtol=0, atol=1e-13)


def test_scale_and_change_of_basis_invariance():
    X, labels, M = random_case(6)
    s, _ = oracle.silhouette_mahalanobis(X, labels, 4, M)
    s2, _ = oracle.silhouette_mahalanobis(X, labels, 4, 7.5 * M)
    np.testing.assert_allclose(s, s2, rtol=0, atol=1e-13)
    A = np.random.default_rng(7).standard_normal((6, 6)) + 3 * np.eye(6)
    Ai = np.linalg.inv(A)
    s3, _ = oracle.silhouette_mahalanobis(X @ A.T, labels, 4, Ai.T @ M @ Ai)
    np.testing.assert_allclose(s, s3, rtol=0, atol=1e-9)


def test_errors():
    X, labels, M = random_case(8, n=10)
    bad = labels.copy()
    bad[3] = 9
    with pytest.raises(oracle.OracleError) as e:
        oracle.silhouette_mahalanobis(X, bad, 4, M)
    assert e.value.code == -3
    with pytest.raises(oracle.OracleError) as e:
        oracle.silhouette_mahalanobis(X, np.zeros(10, np.int32), 4, M)
    assert e.value.code == -4
    X[2, 1] = np.inf
    with pytest.raises(oracle.OracleError) as e:
        oracle.silhouette_mahalanobis(X, labels, 4, M)
    assert e.value.code == -6
