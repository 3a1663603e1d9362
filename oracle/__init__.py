"""FP64 CPU oracle for the linear-complexity Silhouette — TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may import this
package.  The product (the HIP library and its binding) never imports, links or calls it, and
it shares no code with the product.

The arithmetic lives in ``silhouette_oracle.c`` (plain C, binary64, loops in the order of the
paper's equations); this module only marshals numpy arrays through ctypes.

Inputs: ``X`` as a numpy array of float32 / float64, or uint16 (bf16 bit patterns), or uint8
(fp8 e4m3fn codes, with ``col_scale``); ``labels`` int32 in [0, K).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(HERE, "_silhouette_oracle.so")

F32, BF16, FP8_E4M3, F64 = 0, 1, 2, 3
SQEUCLID, COSINE = 0, 1
EUCLID_APPROX = 2  # square roots of the point-to-cluster mean squared distances (Section V)
KL = 3  # generalized Kullback-Leibler divergence of positive vectors (a Bregman divergence)
METRICS = {"sqeuclid": SQEUCLID, "cosine": COSINE, "euclid_approx": EUCLID_APPROX, "kl": KL}

ERRORS = {
    -1: "bad argument",
    -3: "label out of range",
    -4: "fewer than two non-empty clusters",
    -5: "zero-norm point under the cosine distance",
    -6: "non-finite value in X",
    -9: "out of host memory",
    -10: "entry outside the distance's domain (KL needs positive entries)",
}


class OracleError(ValueError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, 'unknown')}")
        self.code = code


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(
            os.path.join(HERE, "silhouette_oracle.c")):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_SO)
    P, I64, I32, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    common = [P, I, P, P, I64, I32, I32, I]
    lib.orc_cluster_stats.argtypes = common + [P, P, P]
    lib.orc_scores_at.argtypes = common + [P, P, P, P, I64, P, P, P, P]
    lib.orc_silhouette.argtypes = common + [P, P, P, P, P]
    lib.orc_brute_silhouette.argtypes = common + [P, P]
    lib.orc_brute_scores_at.argtypes = common + [P, I64, P, P, P]
    lib.orc_gradient.argtypes = common + [P]
    lib.orc_kmeans_step.argtypes = [P, I, P, P, I64, I32, I32, P, P, P, P]
    lib.orc_silhouette_mahalanobis.argtypes = [P, I, P, P, P, I64, I32, I32, P, P, P, P]
    lib.orc_brute_silhouette_mahalanobis.argtypes = [P, I, P, P, P, I64, I32, I32, P, P]
    for f in ("orc_cluster_stats", "orc_scores_at", "orc_silhouette", "orc_brute_silhouette",
              "orc_brute_scores_at", "orc_gradient", "orc_kmeans_step", "orc_silhouette_mahalanobis",
              "orc_brute_silhouette_mahalanobis", "orc_num_threads"):
        getattr(lib, f).restype = ctypes.c_int
    lib.orc_decode_bf16.argtypes = [ctypes.c_uint16]
    lib.orc_decode_bf16.restype = ctypes.c_double
    lib.orc_decode_e4m3.argtypes = [ctypes.c_uint8]
    lib.orc_decode_e4m3.restype = ctypes.c_double
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _prep(X, labels, K, metric, col_scale):
    X = np.ascontiguousarray(X)
    if X.ndim != 2:
        raise ValueError("X must be [N, D]")
    dt = {np.dtype(np.float32): F32, np.dtype(np.float64): F64, np.dtype(np.uint16): BF16,
          np.dtype(np.uint8): FP8_E4M3}.get(X.dtype)
    if dt is None:
        raise TypeError(f"unsupported X dtype {X.dtype}")
    if dt == FP8_E4M3:
        if col_scale is None:
            raise ValueError("fp8 input needs col_scale")
        col_scale = np.ascontiguousarray(col_scale, dtype=np.float32)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    if labels.shape != (X.shape[0],):
        raise ValueError("labels must be [N]")
    m = METRICS[metric] if isinstance(metric, str) else int(metric)
    N, D = X.shape
    return X, dt, col_scale, labels, N, D, int(K), m


def _check(rc):
    if rc != 0:
        raise OracleError(rc)


def cluster_stats(X, labels, K, metric="sqeuclid", col_scale=None):
    """Pass 1 (Eq.5, Eq.6, Eq.8; cosine Eq.15-16): (count int64[K], V f64[K,D], psi f64[K])."""
    X, dt, cs, labels, N, D, K, m = _prep(X, labels, K, metric, col_scale)
    count = np.zeros(K, np.int64)
    V = np.zeros((K, D), np.float64)
    psi = np.zeros(K, np.float64)
    _check(_load().orc_cluster_stats(_ptr(X), dt, _ptr(cs), _ptr(labels), N, D, K, m, _ptr(count),
                                     _ptr(V), _ptr(psi)))
    return count, V, psi


def scores_at(X, labels, K, idx, stats, metric="sqeuclid", col_scale=None):
    """s_i (and a_i, b_i, neighbour id) for the points ``idx`` given pass-1 statistics."""
    X, dt, cs, labels, N, D, K, m = _prep(X, labels, K, metric, col_scale)
    count, V, psi = (np.ascontiguousarray(stats[0], np.int64), np.ascontiguousarray(stats[1], np.float64),
                     np.ascontiguousarray(stats[2], np.float64))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    n = len(idx)
    s, a, b = np.zeros(n), np.zeros(n), np.zeros(n)
    nbr = np.zeros(n, np.int32)
    _check(_load().orc_scores_at(_ptr(X), dt, _ptr(cs), _ptr(labels), N, D, K, m, _ptr(count), _ptr(V),
                                 _ptr(psi), _ptr(idx), n, _ptr(s), _ptr(a), _ptr(b), _ptr(nbr)))
    return s, a, b, nbr


def silhouette(X, labels, K, metric="sqeuclid", col_scale=None, details=False):
    """The paper's linear method in binary64: returns (s f64[N], S) or, with details, also a, b,
    neighbour ids."""
    X, dt, cs, labels, N, D, K, m = _prep(X, labels, K, metric, col_scale)
    s = np.zeros(N)
    S = np.zeros(1)
    a = np.zeros(N) if details else None
    b = np.zeros(N) if details else None
    nbr = np.zeros(N, np.int32) if details else None
    _check(_load().orc_silhouette(_ptr(X), dt, _ptr(cs), _ptr(labels), N, D, K, m, _ptr(s), _ptr(S),
                                  _ptr(a), _ptr(b), _ptr(nbr)))
    if details:
        return s, float(S[0]), a, b, nbr
    return s, float(S[0])


def brute_silhouette(X, labels, K, metric="sqeuclid", col_scale=None):
    """The quadratic definition (all pairwise distances), binary64: (s f64[N], S)."""
    X, dt, cs, labels, N, D, K, m = _prep(X, labels, K, metric, col_scale)
    s = np.zeros(N)
    S = np.zeros(1)
    _check(_load().orc_brute_silhouette(_ptr(X), dt, _ptr(cs), _ptr(labels), N, D, K, m, _ptr(s),
                                        _ptr(S)))
    return s, float(S[0])


def brute_scores_at(X, labels, K, idx, metric="sqeuclid", col_scale=None):
    """The quadratic definition for the points ``idx`` only (each against all N points), binary64:
    (s, a, b) f64[len(idx)]."""
    X, dt, cs, labels, N, D, K, m = _prep(X, labels, K, metric, col_scale)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    n = len(idx)
    s, a, b = np.zeros(n), np.zeros(n), np.zeros(n)
    _check(_load().orc_brute_scores_at(_ptr(X), dt, _ptr(cs), _ptr(labels), N, D, K, m, _ptr(idx), n,
                                       _ptr(s), _ptr(a), _ptr(b)))
    return s, a, b


def gradient(X, labels, K, metric="sqeuclid", col_scale=None):
    """dS/dX (labels fixed), binary64 [N, D]."""
    X, dt, cs, labels, N, D, K, m = _prep(X, labels, K, metric, col_scale)
    dX = np.zeros((N, D))
    _check(_load().orc_gradient(_ptr(X), dt, _ptr(cs), _ptr(labels), N, D, K, m, _ptr(dX)))
    return dX


def _metric_matrix(M, D):
    M = np.ascontiguousarray(M, dtype=np.float64)
    if M.shape != (D, D):
        raise ValueError("M must be [D, D]")
    return M


def silhouette_mahalanobis(X, labels, K, M, col_scale=None, details=False):
    """The linear method under d(x, y) = (x - y)^T M (x - y), binary64: (s f64[N], S) or, with
    details, also a, b."""
    X, dt, cs, labels, N, D, K, _ = _prep(X, labels, K, "sqeuclid", col_scale)
    M = _metric_matrix(M, D)
    s, S = np.zeros(N), np.zeros(1)
    a, b = np.zeros(N), np.zeros(N)
    _check(_load().orc_silhouette_mahalanobis(_ptr(X), dt, _ptr(cs), _ptr(M), _ptr(labels), N, D, K,
                                              _ptr(s), _ptr(S), _ptr(a), _ptr(b)))
    return (s, float(S[0]), a, b) if details else (s, float(S[0]))


def brute_silhouette_mahalanobis(X, labels, K, M, col_scale=None):
    """The quadratic definition under the same distance, binary64: (s f64[N], S)."""
    X, dt, cs, labels, N, D, K, _ = _prep(X, labels, K, "sqeuclid", col_scale)
    M = _metric_matrix(M, D)
    s, S = np.zeros(N), np.zeros(1)
    _check(_load().orc_brute_silhouette_mahalanobis(_ptr(X), dt, _ptr(cs), _ptr(M), _ptr(labels), N, D, K,
                                                    _ptr(s), _ptr(S)))
    return s, float(S[0])


def kmeans_step(X, labels, K, col_scale=None):
    """One Lloyd step (means from `labels`, then nearest non-empty mean, lowest id on ties),
    binary64: (new labels int32[N], inertia, d1 f64[N] distance to the chosen mean, d2 f64[N]
    next smallest distance, +inf when there is none)."""
    X, dt, cs, labels, N, D, K, _ = _prep(X, labels, K, "sqeuclid", col_scale)
    out = np.zeros(N, np.int32)
    inertia = np.zeros(1)
    d1, d2 = np.zeros(N), np.zeros(N)
    _check(_load().orc_kmeans_step(_ptr(X), dt, _ptr(cs), _ptr(labels), N, D, K, _ptr(out),
                                   _ptr(inertia), _ptr(d1), _ptr(d2)))
    return out, float(inertia[0]), d1, d2


def decode_bf16(bits: int) -> float:
    return _load().orc_decode_bf16(int(bits))


def decode_e4m3(code: int) -> float:
    return _load().orc_decode_e4m3(int(code))


def num_threads() -> int:
    return _load().orc_num_threads()
