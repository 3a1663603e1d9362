"""The C-ABI library loads and exports every entry point include/silhouette.h declares, and the
host-side argument checks behave as documented (no device work is launched here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "silhouette.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(silhouette_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2303_14102_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsilhouette.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("silhouette_sqeuclid", "silhouette_cosine", "silhouette_workspace_bytes",
              "silhouette_cluster_stats", "silhouette_status", "silhouette_strerror"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2303_14102_amd import _lib
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"


def test_workspace_bytes_host_logic(lib):
    from paper_2303_14102_amd import _lib
    f = lib.silhouette_workspace_bytes
    assert f(0, 8, 4, 0, 0, 0) == 0
    assert f(10, 0, 4, 0, 0, 0) == 0
    assert f(10, 257, 4, 0, 0, 0) == 0
    assert f(10, 8, 1, 0, 0, 0) == 0
    assert f(10, 8, 65537, 0, 0, 0) == 0
    a = f(10_000, 8, 4, 0, _lib.SIL_F32, 0)
    b = f(10_000, 8, 4, 0, _lib.SIL_F32, _lib.SIL_FLAG_SAVE_FOR_GRAD)
    assert a > 0 and b >= a + 3 * 4 * 10_000
    # grows linearly in N (sorted row ids and labels: 8 bytes a point), plus tables independent of N
    big = f(50_000_000, 128, 1000, 0, _lib.SIL_F32, 0)
    assert 50_000_000 * 8 < big < 50_000_000 * 8 + 64 * 2**20
    # squared Euclidean with bf16 storage adds the one-product screen's list of fallback rows
    big = f(50_000_000, 128, 1000, 0, _lib.SIL_BF16, 0)
    assert 50_000_000 * 12 < big < 50_000_000 * 12 + 64 * 2**20
    assert f(50_000_000, 128, 1000, 0, _lib.SIL_BF16, _lib.SIL_FLAG_NO_SCREEN) < 50_000_000 * 8 + 64 * 2**20
    assert f(2**31 - 1, 1, 2, 0, 0, 0) > 0
    assert f(2**31, 1, 2, 0, 0, 0) == 0


def test_host_argument_errors_launch_nothing(lib):
    from paper_2303_14102_amd import _lib
    fake = ctypes.c_void_p(0x1000)       # never dereferenced: every call below fails its checks first
    ws = ctypes.c_void_p(0x100000)
    for fn in (lib.silhouette_sqeuclid, lib.silhouette_cosine):
        assert fn(None, 0, None, fake, 10, 4, 2, 0, 0, None, fake, ws, 1 << 30, None) == -1
        assert fn(fake, 0, None, None, 10, 4, 2, 0, 0, None, fake, ws, 1 << 30, None) == -1
        assert fn(fake, 0, None, fake, 0, 4, 2, 0, 0, None, fake, ws, 1 << 30, None) == -1
        assert fn(fake, 0, None, fake, 10, 4, 1, 0, 0, None, fake, ws, 1 << 30, None) == -1
        assert fn(fake, 7, None, fake, 10, 4, 2, 0, 0, None, fake, ws, 1 << 30, None) == -2
        assert fn(fake, 2, None, fake, 10, 4, 2, 0, 0, None, fake, ws, 1 << 30, None) == -2  # fp8 w/o scale
        assert fn(fake, 0, None, fake, 10, 4, 2, 0, 0, None, fake, ws, 16, None) == -7       # too small
        assert fn(fake, 0, None, fake, 10, 4, 2, 0, 0, None, fake, ctypes.c_void_p(0x100010), 1 << 30, None) == -7
        assert fn(fake, 0, None, fake, 10, 4, 2, 0, 0, None, fake, None, 1 << 30, None) == -7
        assert fn(fake, 0, None, fake, 10, 4, 2, 4, 0, None, fake, ws, 1 << 30, None) == -1  # products
        assert fn(fake, 0, None, fake, 10, 4, 2, 0, 0, None, None, ws, 1 << 30, None) == -1  # S NULL
        # backward saves exist for fp32 storage only
        assert fn(fake, 1, None, fake, 10, 4, 2, 0, _lib.SIL_FLAG_SAVE_FOR_GRAD, None, fake, ws, 1 << 30, None) == -2
        # the approximate Euclidean form has no backward
        approx_save = _lib.SIL_FLAG_EUCLID_APPROX | _lib.SIL_FLAG_SAVE_FOR_GRAD
        assert fn(fake, 0, None, fake, 10, 4, 2, 0, approx_save, None, fake, ws, 1 << 30, None) == -1
        # X at an address that is not 16-byte aligned
        odd = ctypes.c_void_p(0x1004)
        assert fn(odd, 0, None, fake, 10, 4, 2, 0, 0, None, fake, ws, 1 << 30, None) == -1
    # ... and is a squared Euclidean form
    assert lib.silhouette_cosine(fake, 0, None, fake, 10, 4, 2, 0, _lib.SIL_FLAG_EUCLID_APPROX, None, fake, ws,
                                 1 << 30, None) == -1
    for bw in (lib.silhouette_sqeuclid_backward, lib.silhouette_cosine_backward):
        assert bw(fake, 0, None, fake, 10, 4, 2, _lib.SIL_FLAG_EUCLID_APPROX, fake, fake, ws, 1 << 30, None) == -1


def test_kmeans_host_checks(lib):
    from paper_2303_14102_amd import _lib
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x100000)
    f = lib.silhouette_kmeans_step
    # (X, dtype, col_scale, labels, N, D, K, products, flags, labels_out, inertia, ws, bytes, stream)
    assert f(fake, 0, None, fake, 10, 4, 2, 0, _lib.SIL_FLAG_SAVE_FOR_GRAD, fake, fake, ws, 1 << 30, None) == -1
    assert f(fake, 0, None, fake, 10, 4, 2, 0, _lib.SIL_FLAG_EUCLID_APPROX, fake, fake, ws, 1 << 30, None) == -1
    assert f(fake, 1, None, fake, 10, 4, 2, 1, 0, fake, fake, ws, 1 << 30, None) == -1   # products
    assert f(fake, 0, None, fake, 10, 4, 2, 2, 0, fake, fake, ws, 1 << 30, None) == -1   # 2: bf16 only
    assert f(fake, 2, fake, fake, 10, 4, 2, 2, 0, fake, fake, ws, 1 << 30, None) == -1
    assert f(fake, 0, None, fake, 10, 4, 2, 0, 0, None, fake, ws, 1 << 30, None) == -1   # labels_out
    assert f(fake, 0, None, fake, 10, 4, 2, 0, 0, fake, None, ws, 1 << 30, None) == -1   # inertia
    assert f(fake, 0, None, fake, 10, 4, 1, 0, 0, fake, fake, ws, 1 << 30, None) == -1   # K
    assert f(fake, 2, None, fake, 10, 4, 2, 0, 0, fake, fake, ws, 1 << 30, None) == -2   # fp8 w/o scale
    assert f(fake, 0, None, fake, 10, 4, 2, 0, 0, fake, fake, ws, 16, None) == -7        # workspace


def test_stream_host_checks(lib):
    from paper_2303_14102_amd import _lib
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x100000)
    f = lib.silhouette_stream
    # (metric, X, dtype, col_scale, labels, N, D, K, products, flags, s, S, chunk, ws, bytes, stream)
    assert f(0, fake, 0, None, fake, 100, 4, 2, 0, 0, None, fake, 0, ws, 1 << 30, None) == -1     # chunk
    assert f(0, None, 0, None, fake, 100, 4, 2, 0, 0, None, fake, 10, ws, 1 << 30, None) == -1    # X
    assert f(0, fake, 0, None, fake, 100, 4, 2, 0, 0, None, None, 10, ws, 1 << 30, None) == -1    # S
    assert f(2, fake, 0, None, fake, 100, 4, 2, 0, 0, None, fake, 10, ws, 1 << 30, None) == -1    # metric
    assert f(1, fake, 0, None, fake, 100, 4, 2, 0, _lib.SIL_FLAG_EUCLID_APPROX, None, fake, 10, ws, 1 << 30,
             None) == -1
    assert f(0, fake, 0, None, fake, 100, 4, 2, 0, _lib.SIL_FLAG_SAVE_FOR_GRAD, None, fake, 10, ws, 1 << 30,
             None) == -1
    assert f(0, fake, 2, None, fake, 100, 4, 2, 0, 0, None, fake, 10, ws, 1 << 30, None) == -2    # fp8 scale
    assert f(0, fake, 0, None, fake, 100, 4, 2, 0, 0, None, fake, 10, ws, 16, None) == -7         # workspace
    sz = lib.silhouette_stream_workspace_bytes
    assert sz(100, 0, 4, 2, 0, 0, 0) == 0
    a, b = sz(10_000, 1_000, 8, 4, 0, 0, 0), sz(10_000, 2_000, 8, 4, 0, 0, 0)
    assert 0 < a < b  # two chunk buffers grow with the chunk
    assert sz(10_000, 20_000, 8, 4, 0, 0, 0) == sz(10_000, 10_000, 8, 4, 0, 0, 0)  # clamped to N


def test_mahalanobis_host_checks(lib):
    from paper_2303_14102_amd import _lib
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x100000)
    f = lib.silhouette_mahalanobis
    # (X, dtype, col_scale, L, labels, N, D, K, flags, s, S, ws, bytes, stream)
    assert f(fake, 0, None, None, fake, 10, 4, 2, 0, None, fake, ws, 1 << 30, None) == -1   # L
    assert f(fake, 0, None, fake, fake, 10, 4, 2, _lib.SIL_FLAG_EUCLID_APPROX, None, fake, ws, 1 << 30, None) == -1
    assert f(fake, 0, None, fake, fake, 10, 4, 2, 0, None, None, ws, 1 << 30, None) == -1   # S
    assert f(fake, 2, None, fake, fake, 10, 4, 2, 0, None, fake, ws, 1 << 30, None) == -2   # fp8 scale
    assert f(fake, 0, None, fake, fake, 10, 4, 2, 0, None, fake, ws, 64, None) == -7        # workspace
    assert f(ctypes.c_void_p(0x1004), 0, None, fake, fake, 10, 4, 2, 0, None, fake, ws, 1 << 30, None) == -1
    sz = lib.silhouette_mahalanobis_workspace_bytes
    assert sz(1000, 8, 4, 0) >= 1000 * 8 * 4 + lib.silhouette_workspace_bytes(1000, 8, 4, 0, 0, 0)
    assert sz(0, 8, 4, 0) == 0


def test_kl_host_checks(lib):
    from paper_2303_14102_amd import _lib
    fake = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x100000)
    f = lib.silhouette_kl
    assert f(fake, 2, fake, fake, 10, 4, 2, 0, 0, None, fake, ws, 1 << 30, None) == -2   # fp8
    assert f(fake, 0, None, fake, 10, 4, 2, 0, _lib.SIL_FLAG_SAVE_FOR_GRAD, None, fake, ws, 1 << 30, None) == -1
    assert f(fake, 0, None, fake, 10, 4, 2, 0, _lib.SIL_FLAG_EUCLID_APPROX, None, fake, ws, 1 << 30, None) == -1
    assert f(fake, 0, None, fake, 10, 4, 2, 4, 0, None, fake, ws, 1 << 30, None) == -1   # products
    assert f(fake, 0, None, fake, 10, 4, 2, 0, 0, None, fake, ws, 16, None) == -7        # workspace
    assert lib.silhouette_workspace_bytes(100, 8, 4, _lib.SIL_KL, 0, 0) > 0


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10, 99):
        assert isinstance(lib.silhouette_strerror(code), bytes)


def test_batched_plan_host_checks(lib):
    # descriptor checks happen before any device query; nothing is launched
    from paper_2303_14102_amd import _lib
    fake = 0x1000

    def plan(probs, flags=0):
        arr = (_lib.SilProblem * max(1, len(probs)))(*probs)
        out = ctypes.c_void_p(123)
        rc = lib.silhouette_batched_plan(arr, len(probs), flags, ctypes.byref(out))
        assert out.value is None  # no plan on failure
        return rc

    ok = dict(X=fake, labels=fake, N=100, D=16, K=4, dtype=_lib.SIL_F32, metric=0, s=0, S=fake)

    def P(**kw):
        return _lib.SilProblem(**{**ok, **kw})

    assert plan([]) == -1                                   # no problems
    assert plan([P()] * 1025) == -1                         # too many
    assert plan([P(D=129)]) == -1                           # deeper than the batched kernel
    assert plan([P(D=0)]) == -1
    assert plan([P(K=1)]) == -1
    assert plan([P(K=16385)]) == -1
    assert plan([P(N=0)]) == -1
    assert plan([P(N=2**31)]) == -1
    assert plan([P(metric=2)]) == -1
    assert plan([P(X=0)]) == -1
    assert plan([P(X=fake + 4)]) == -1                      # X not 16-byte aligned
    assert plan([P(labels=0)]) == -1
    assert plan([P(S=0)]) == -1
    assert plan([P(), P(dtype=_lib.SIL_BF16)]) == -2        # fp32 storage only
    assert plan([P()], flags=_lib.SIL_FLAG_SAVE_FOR_GRAD) == -1
    assert plan([P()], flags=1 << 3) == -1                  # unknown flag bit
    assert lib.silhouette_batched_plan(None, 1, 0, ctypes.byref(ctypes.c_void_p())) == -1
    # valid descriptors: without a GPU the plan fails at its device query (SIL_E_HIP) and frees
    # what it built; with one it is created (nothing is launched) and freed here
    arr = (_lib.SilProblem * 3)(P(), P(D=64, K=300), P(D=128, K=2, metric=1))
    out = ctypes.c_void_p()
    rc = lib.silhouette_batched_plan(arr, 3, 0, ctypes.byref(out))
    assert rc in (0, -8)
    if rc == 0:
        assert lib.silhouette_batched_workspace_bytes(out) > 0
        lib.silhouette_batched_free(out)
    else:
        assert out.value is None
    assert lib.silhouette_batched_workspace_bytes(None) == 0
    assert lib.silhouette_batched_run(None, ctypes.c_void_p(fake), 1, None) == -1
    assert lib.silhouette_batched_replay(None, None) == -1
    assert lib.silhouette_batched_set_config(None, None, 6) == -1
    lib.silhouette_batched_free(None)


def test_fp8_col_scale_checks_on_the_host():
    """fp8 storage: col_scale must be a contiguous float32 [D] tensor on X's device; anything
    else raises before a pointer reaches the C ABI."""
    import torch

    from paper_2303_14102_amd import binding as sil
    cpu = torch.device("cpu")
    good = torch.ones(8, dtype=torch.float32)
    sil._check_col_scale(good, 8, cpu)
    bad = [None, good.double(), torch.ones(9), torch.ones(16)[::2], torch.ones(8, 1).squeeze(1)[:7],
           torch.ones(8, device="meta")]
    for cs in bad:
        with pytest.raises(ValueError):
            sil._check_col_scale(cs, 8, cpu)
