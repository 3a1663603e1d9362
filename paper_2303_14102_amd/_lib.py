"""ctypes binding of libsilhouette.so (the HIP library built from csrc/).

Argument marshalling only: every step of the computation runs in the library's kernels.  The
library is loaded from this package directory; if it is missing the import fails loudly (build
it with ``python -m paper_2303_14102_amd.build``).  There is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# SIL_LIBRARY names another build of the same library (the AddressSanitizer host build, for one)
LIB_PATH = os.environ.get("SIL_LIBRARY") or os.path.join(HERE, "libsilhouette.so")

SIL_OK = 0
STATUS = {
    0: "SIL_OK", -1: "SIL_E_ARG", -2: "SIL_E_DTYPE", -3: "SIL_E_LABEL", -4: "SIL_E_FEW_CLUSTERS",
    -5: "SIL_E_ZERO_NORM", -6: "SIL_E_NONFINITE", -7: "SIL_E_WORKSPACE", -8: "SIL_E_HIP",
    -9: "SIL_E_DOMAIN", -10: "SIL_E_SCRATCH",
}
SIL_NOALLOC_SCRATCH_BYTES = 64 << 20
SIL_F32, SIL_BF16, SIL_FP8_E4M3 = 0, 1, 2
SIL_SQEUCLID, SIL_COSINE, SIL_KL = 0, 1, 2
SIL_FLAG_NO_CENTRE = 1 << 0
SIL_FLAG_SAVE_FOR_GRAD = 1 << 1
SIL_FLAG_EUCLID_APPROX = 1 << 2
SIL_FLAG_NO_SCREEN = 1 << 3

# every symbol include/silhouette.h declares, with its ctypes signature
_P, _I32, _I64, _SZ, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
SIGNATURES = {
    "silhouette_workspace_bytes": (_SZ, [_I64, _I32, _I32, _I32, _I32, _I32]),
    "silhouette_sqeuclid": (ctypes.c_int, [_P, _I32, _P, _P, _I64, _I32, _I32, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "silhouette_sqeuclid_noalloc": (ctypes.c_int, [_P, _I32, _P, _P, _I64, _I32, _I32, _I32, _I32, _P, _P, _P, _P]),
    "silhouette_cosine": (ctypes.c_int, [_P, _I32, _P, _P, _I64, _I32, _I32, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "silhouette_kl": (ctypes.c_int, [_P, _I32, _P, _P, _I64, _I32, _I32, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "silhouette_cluster_stats": (ctypes.c_int, [_P, _I32, _P, _P, _I64, _I32, _I32, _I32, _P, _P, _P, _P, _SZ, _P]),
    "silhouette_stream_workspace_bytes": (_SZ, [_I64, _I64, _I32, _I32, _I32, _I32, _I32]),
    "silhouette_stream": (ctypes.c_int, [_I32, _P, _I32, _P, _P, _I64, _I32, _I32, _I32, _I32, _P, _P, _I64, _P, _SZ, _P]),
    "silhouette_mahalanobis_workspace_bytes": (_SZ, [_I64, _I32, _I32, _I32]),
    "silhouette_mahalanobis": (ctypes.c_int, [_P, _I32, _P, _P, _P, _I64, _I32, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "silhouette_kmeans_step": (ctypes.c_int, [_P, _I32, _P, _P, _I64, _I32, _I32, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "silhouette_status": (ctypes.c_int, [_P, _P]),
    "silhouette_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "silhouette_sqeuclid_backward": (ctypes.c_int, [_P, _I32, _P, _P, _I64, _I32, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "silhouette_cosine_backward": (ctypes.c_int, [_P, _I32, _P, _P, _I64, _I32, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "silhouette_profile_begin": (ctypes.c_int, [_I32]),
    "silhouette_profile_end": (ctypes.c_int, [_P, _P]),
    "silhouette_batched_plan": (ctypes.c_int, [_P, _I32, _I32, _P]),
    "silhouette_batched_workspace_bytes": (_SZ, [_P]),
    "silhouette_batched_run": (ctypes.c_int, [_P, _P, _SZ, _P]),
    "silhouette_batched_tune": (ctypes.c_int, [_P, _P, _SZ, _P, _P]),
    "silhouette_batched_config": (ctypes.c_int, [_P, _P, _I32]),
    "silhouette_batched_set_config": (ctypes.c_int, [_P, _P, _I32]),
    "silhouette_batched_capture": (ctypes.c_int, [_P, _P, _SZ, _P]),
    "silhouette_batched_replay": (ctypes.c_int, [_P, _P]),
    "silhouette_batched_status": (ctypes.c_int, [_P, _P, _P, _P]),
    "silhouette_batched_free": (None, [_P]),
}


class SilProblem(ctypes.Structure):
    """struct sil_problem of include/silhouette.h."""
    _fields_ = [("X", _P), ("labels", _P), ("N", _I64), ("D", _I32), ("K", _I32), ("dtype", _I32),
                ("metric", _I32), ("s", _P), ("S", _P)]


class SilhouetteError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)} ({strerror(code)})")


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2303_14102_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def strerror(code: int) -> str:
    return load().silhouette_strerror(int(code)).decode()


def check(code: int, where: str) -> None:
    if code != SIL_OK:
        raise SilhouetteError(code, where)
