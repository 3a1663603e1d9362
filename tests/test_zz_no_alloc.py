"""silhouette_sqeuclid_noalloc, the entry point for callers that cannot allocate (its workspace
is the library's static per-GPU scratch), through the C ABI: two calls in a row, the second on a
smaller problem, each against silhouette_sqeuclid with a caller workspace on the same inputs and
against the FP64 oracle; the size limit and the flag it refuses are host errors."""

import ctypes
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


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def test_noalloc_matches_workspace_entry_point(dev):
    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    lib = _lib.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    # (N, D, K, form, products, seed, singletons): the larger problem first, then a smaller one,
    # so the second call runs on scratch that still holds the first call's data
    cases = [(150_001, 64, 300, "bf16", 2, 81, 2), (40_003, 40, 37, "f32", 0, 82, 1)]
    for n, d, k, form, products, seed, single in cases:
        b = wl.make_small(n, d, k, seed=seed, singletons=single)
        X, cs, codes = storage(b.X.to(dev), form)
        lab = b.labels.to(dev)
        lab_h = b.labels.numpy()
        print(f"[noalloc] N={n} D={d} K={k} {form} products={products}", flush=True)
        s1 = torch.full((n,), float("nan"), dtype=torch.float32, device=dev)
        S1 = torch.full((), float("nan"), dtype=torch.float64, device=dev)
        st = torch.full((1,), 12345, dtype=torch.int32, device=dev)
        rc = lib.silhouette_sqeuclid_noalloc(_p(X), sil._dtype_code(X), _p(cs), _p(lab), n, d, k, products, 0,
                                             _p(s1), _p(S1), _p(st), stream)
        assert rc == 0, _lib.strerror(rc)
        ws = sil.new_workspace(n, d, k, "sqeuclid", X.dtype, 0, dev)
        s2 = torch.empty(n, dtype=torch.float32, device=dev)
        S2 = torch.empty((), dtype=torch.float64, device=dev)
        rc = lib.silhouette_sqeuclid(_p(X), sil._dtype_code(X), _p(cs), _p(lab), n, d, k, products, 0,
                                     _p(s2), _p(S2), _p(ws), ws.numel(), stream)
        assert rc == 0, _lib.strerror(rc)
        torch.cuda.synchronize()
        assert int(st.item()) == 0 and sil.status(ws) == 0
        s_ref, S_ref, a, bb, _ = oracle.silhouette(codes, lab_h, k, "sqeuclid", details=True)
        bound = per_point_bound(form, products, "sqeuclid", True, dequantised(codes, None), lab_h, k, a, bb)
        sa, sb = s1.cpu().numpy().astype(np.float64), s2.cpu().numpy().astype(np.float64)
        print(f"  S noalloc={S1.item():.12f} workspace={S2.item():.12f} oracle={S_ref:.12f} "
              f"max|s_noalloc - s_ws|={np.abs(sa - sb).max():.2e}", flush=True)
        assert np.all(np.abs(sa - s_ref) <= bound)
        assert np.all(np.abs(sb - s_ref) <= bound)
        assert np.all(np.abs(sa - sb) <= 2 * bound)
        assert abs(S1.item() - S_ref) <= TOL_S_MEAN[form]
        assert abs(S1.item() - S2.item()) <= TOL_S_MEAN[form]


def test_noalloc_binding_and_device_error(dev):
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(5_000, 16, 6, seed=83)
    X, lab = b.X.to(dev), b.labels.to(dev)
    s = torch.empty(5_000, dtype=torch.float32, device=dev)
    S = torch.empty((), dtype=torch.float64, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    sil.sqeuclid_noalloc(X, lab, 6, s=s, S=S, status=st)
    s_ref, S_ref = oracle.silhouette(b.X.numpy(), b.labels.numpy(), 6, "sqeuclid")
    torch.cuda.synchronize()
    assert st.item() == 0 and abs(S.item() - S_ref) <= TOL_S_MEAN["f32"]
    bad = lab.clone()
    bad[11] = 6  # a label outside [0, K): found on the device, S and s become NaN
    sil.sqeuclid_noalloc(X, bad, 6, s=s, S=S, status=st)
    torch.cuda.synchronize()
    assert st.item() == -3 and math.isnan(S.item()) and torch.isnan(s).all()
    # and the next good call on the same scratch is clean again
    sil.sqeuclid_noalloc(X, lab, 6, s=s, S=S, status=st)
    torch.cuda.synchronize()
    assert st.item() == 0 and abs(S.item() - S_ref) <= TOL_S_MEAN["f32"]


def test_noalloc_host_limits(dev):
    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    lib = _lib.load()
    X = torch.zeros(16, 8, device=dev)
    lab = torch.zeros(16, dtype=torch.int32, device=dev)
    S = torch.full((), 7.0, dtype=torch.float64, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    # a shape whose workspace exceeds the scratch: refused on the host before anything reads X
    big_n = 10_000_000
    assert lib.silhouette_workspace_bytes(big_n, 8, 4, 0, 0, 0) > _lib.SIL_NOALLOC_SCRATCH_BYTES
    rc = lib.silhouette_sqeuclid_noalloc(_p(X), 0, None, _p(lab), big_n, 8, 4, 0, 0, None, _p(S), None, stream)
    assert rc == -10 and "scratch" in _lib.strerror(rc)
    rc = lib.silhouette_sqeuclid_noalloc(_p(X), 0, None, _p(lab), 16, 8, 4, 0, _lib.SIL_FLAG_SAVE_FOR_GRAD,
                                         None, _p(S), None, stream)
    assert rc == -1
    rc = lib.silhouette_sqeuclid_noalloc(_p(X), 0, None, _p(lab), 16, 8, 4, 0, 0, None, None, None, stream)
    assert rc == -1
    torch.cuda.synchronize()
    assert S.item() == 7.0  # nothing ran
    with pytest.raises(ValueError):
        sil.sqeuclid_noalloc(X, lab, 4, s=torch.empty(15, device=dev))
