"""dS/dX from the HIP backward (through the C ABI and the autograd Function) against the FP64
oracle's gradient and against central finite differences of the oracle's S.

Tolerance: relative L2 error <= 1e-4 over the compared entries (the gradient is formed in fp32
from fp32 statistics; S itself is within 1e-6)."""

import numpy as np
import pytest
import torch

import oracle
from paper_2303_14102_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_14102_amd import _lib
    _lib.load()
    return torch.device("cuda:0")


def rel_l2(g, ref):
    return float(np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300))


def kink_rows(X, labels, K, metric, rel=1e-4):
    """Rows whose two nearest other clusters are within `rel` (relative) of each other in binary64
    (mean distances from the oracle's cluster statistics, Eq.11 / Eq.18).  There s_i is a minimum
    of two nearly equal terms: the fp32 forward may take either as the neighbour (its error in b
    is below 1e-6 relative on these workloads), and dS/dx_i is a different one-sided derivative
    for each, so such rows have no unique gradient to compare."""
    count, V, psi = oracle.cluster_stats(X, labels, K, metric)
    Xd = X.astype(np.float64)
    nk = np.maximum(count, 1).astype(np.float64)
    if metric == "cosine":
        Z = Xd / np.linalg.norm(Xd, axis=1)[:, None]
        d = 1.0 - Z @ (V / nk[:, None]).T
    else:
        d = (Xd * Xd).sum(1)[:, None] - 2.0 * Xd @ (V / nk[:, None]).T + (psi / nk)[None, :]
    d[:, count == 0] = np.inf
    d[np.arange(len(labels)), labels] = np.inf
    two = np.partition(d, 1, axis=1)[:, :2]
    return (two[:, 1] - two[:, 0]) <= rel * np.abs(two[:, 0])


def gpu_grad(dev, X, labels, K, metric):
    from paper_2303_14102_amd import binding as sil
    Xd = X.to(dev).requires_grad_(True)
    S = sil.SilhouetteFn.apply(Xd, labels.to(dev), K, metric)
    S.backward()
    torch.cuda.synchronize()
    return S.item(), Xd.grad.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
# (4000, 256, 64) and (3000, 256, 79) keep their K (D+1) FP64 partials in LDS (131.6 and
# 162.4 KB of the 160 KB budget)
@pytest.mark.parametrize("n,d,k,single", [(2000, 16, 7, 1), (3001, 40, 33, 2), (4000, 256, 64, 0),
                                          (3000, 256, 79, 1)])
def test_gradient_vs_oracle(dev, metric, n, d, k, single):
    b = wl.make_small(n, d, k, seed=31 + d, singletons=single, sigma=1.5)
    print(f"[bwd] metric={metric} N={n} D={d} K={k}", flush=True)
    S, g = gpu_grad(dev, b.X, b.labels, k, metric)
    ref = oracle.gradient(b.X.numpy(), b.labels.numpy(), k, metric)
    _, S_ref = oracle.silhouette(b.X.numpy(), b.labels.numpy(), k, metric)
    err = rel_l2(g, ref)
    print(f"  S={S:.9f} ref={S_ref:.9f} rel_l2(dX)={err:.2e}", flush=True)
    assert abs(S - S_ref) <= 1e-6
    assert err <= 1e-4


# the accumulation forms: squared Euclidean by 64-column slices (K x 65 partials in LDS, here
# 104 KB and 41.6 KB), and global atomics once neither K x 65 nor K (D+1) FP64 values fit the
# 160 KB budget (squared Euclidean K = 320, D = 64; cosine K = 80, D = 256)
@pytest.mark.parametrize("n,d,k,metric", [(6000, 128, 200, "sqeuclid"), (3000, 256, 80, "sqeuclid"),
                                          (5000, 64, 320, "sqeuclid"), (3000, 256, 80, "cosine")])
def test_gradient_accumulation_paths(dev, n, d, k, metric):
    b = wl.make_small(n, d, k, seed=41, sigma=1.0)
    S, g = gpu_grad(dev, b.X, b.labels, k, metric)
    ref = oracle.gradient(b.X.numpy(), b.labels.numpy(), k, metric)
    assert rel_l2(g, ref) <= 1e-4


# the two dX kernels: four columns per lane (D % 4 == 0, D > 128; at D = 132 lanes 33..63 idle)
# and one column per lane (D = 201; and D = 256 when dX is only 4-byte aligned)
@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
@pytest.mark.parametrize("n,d,k,offset", [(2500, 132, 9, 0), (2500, 201, 9, 0), (2500, 256, 9, 1)])
def test_gradient_dx_forms(dev, metric, n, d, k, offset):
    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(n, d, k, seed=53 + d, singletons=1, sigma=1.2)
    print(f"[bwd-dx] metric={metric} N={n} D={d} K={k} offset={offset}", flush=True)
    lib = _lib.load()
    flags = _lib.SIL_FLAG_SAVE_FOR_GRAD
    m = 0 if metric == "sqeuclid" else 1
    # dX at a 4-byte offset into its buffer when offset = 1 (X itself must be 16-byte aligned)
    X = b.X.to(dev).contiguous()
    gbuf = torch.zeros(n * d + offset, dtype=torch.float32, device=dev)
    dX = gbuf[offset:].view(n, d)
    lab = b.labels.to(dev)
    ws = sil.new_workspace(n, d, k, metric, torch.float32, flags, dev)
    S = torch.empty((), dtype=torch.float64, device=dev)
    gS = torch.ones((), dtype=torch.float64, device=dev)
    st = sil._stream(dev)
    fwd = lib.silhouette_sqeuclid if m == 0 else lib.silhouette_cosine
    bwd = lib.silhouette_sqeuclid_backward if m == 0 else lib.silhouette_cosine_backward
    _lib.check(fwd(sil._ptr(X), 0, None, sil._ptr(lab), n, d, k, 0, flags, None, sil._ptr(S),
                   sil._ptr(ws), ws.numel(), st), "forward")
    _lib.check(bwd(sil._ptr(X), 0, None, sil._ptr(lab), n, d, k, flags, sil._ptr(gS), sil._ptr(dX),
                   sil._ptr(ws), ws.numel(), st), "backward")
    torch.cuda.synchronize()
    ref = oracle.gradient(b.X.numpy(), b.labels.numpy(), k, metric)
    err = rel_l2(dX.cpu().numpy().astype(np.float64), ref)
    print(f"  rel_l2(dX)={err:.2e}", flush=True)
    assert err <= 1e-4


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
def test_gradient_vs_finite_differences(dev, metric):
    # central differences (h = 1e-3) of the FP64 oracle's S on 64 sampled coordinates away from
    # kinks (|a - b| not small), against the GPU gradient
    b = wl.make_small(20_000, 32, 10, seed=5, sigma=1.5)
    X = b.X.numpy().astype(np.float64)
    lab = b.labels.numpy()
    _, g = gpu_grad(dev, b.X, b.labels, 10, metric)
    _, _, a, bb, _ = oracle.silhouette(X, lab, 10, metric, details=True)
    ok = np.flatnonzero(np.abs(a - bb) > 0.2 * np.maximum(a, bb))
    rng = np.random.default_rng(5)
    rows = rng.choice(ok, size=64, replace=False)
    cols = rng.integers(0, X.shape[1], size=64)
    h = 1e-3
    fd = np.empty(64)
    for t, (i, l) in enumerate(zip(rows, cols)):
        Xp, Xm = X.copy(), X.copy()
        Xp[i, l] += h
        Xm[i, l] -= h
        fd[t] = (oracle.silhouette(Xp, lab, 10, metric)[1] - oracle.silhouette(Xm, lab, 10, metric)[1]) / (2 * h)
    got = g[rows, cols]
    err = rel_l2(got, fd)
    print(f"  FD rel_l2={err:.2e} max|fd|={np.abs(fd).max():.3e}", flush=True)
    assert err <= 1e-4


def test_gradient_flows_through_autograd(dev):
    # S as a loss inside a torch graph: d(3 S + 1)/dX = 3 dS/dX
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(1500, 8, 5, seed=9)
    Xd = b.X.to(dev).requires_grad_(True)
    (3.0 * sil.SilhouetteFn.apply(Xd, b.labels.to(dev), 5, "sqeuclid") + 1.0).backward()
    ref = oracle.gradient(b.X.numpy(), b.labels.numpy(), 5, "sqeuclid")
    assert rel_l2(Xd.grad.cpu().numpy().astype(np.float64), 3.0 * ref) <= 1e-4


@pytest.mark.parametrize("metric", ["sqeuclid", "cosine"])
def test_gradient_full_size_workload(dev, metric):
    # the differentiation workload at its full size: N = 1e6 points, D = 256, K = 64
    from paper_2303_14102_amd import binding as sil
    spec = wl.WORKLOADS["blobs-1m-d256-k64"]
    b = wl.make_blobs(spec, dev)
    print(f"[bwd-full] {spec.name} {metric}", flush=True)
    Xd = b.X.requires_grad_(True)
    S = sil.SilhouetteFn.apply(Xd, b.labels, spec.k, metric)
    S.backward()
    torch.cuda.synchronize()
    g = Xd.grad.cpu().numpy().astype(np.float64)
    Xh = b.X.detach().cpu().numpy()
    lab = b.labels.cpu().numpy()
    ref = oracle.gradient(Xh, lab, spec.k, metric)
    kink = kink_rows(Xh, lab, spec.k, metric)
    err_all, err = rel_l2(g, ref), rel_l2(g[~kink], ref[~kink])
    print(f"  rel_l2(dX)={err:.2e} over {int((~kink).sum())} rows ({err_all:.2e} with the "
          f"{int(kink.sum())} rows at a kink)", flush=True)
    assert kink.mean() < 0.005
    assert err <= 1e-4


def test_gradient_full_size_finite_differences(dev):
    # the differentiation workload at its full size (N = 1e6, D = 256, K = 64) against central
    # differences (h = 1e-3) of the FP64 oracle's S along 8 directions, each touching 8 sampled
    # coordinates (distinct rows away from kinks, |a - b| > 0.2 max(a, b)) with signs +-1.
    # Each difference of S is summed from the per-point differences s_j(X + hU) - s_j(X - hU),
    # so the rounding of the two S values (sums of 1e6 terms) does not enter it.
    from paper_2303_14102_amd import binding as sil
    spec = wl.WORKLOADS["blobs-1m-d256-k64"]
    b = wl.make_blobs(spec, dev)
    print(f"[bwd-fd-full] {spec.name}", flush=True)
    Xd = b.X.requires_grad_(True)
    S = sil.SilhouetteFn.apply(Xd, b.labels, spec.k, "sqeuclid")
    S.backward()
    torch.cuda.synchronize()
    g = Xd.grad.cpu().numpy().astype(np.float64)
    X = b.X.detach().cpu().numpy().astype(np.float64)
    lab = b.labels.cpu().numpy()
    _, _, a, bb, _ = oracle.silhouette(X, lab, spec.k, details=True)
    ok = np.flatnonzero(np.abs(a - bb) > 0.2 * np.maximum(a, bb))
    rng = np.random.default_rng(17)
    rows = rng.choice(ok, size=64, replace=False).reshape(8, 8)
    cols = rng.integers(0, X.shape[1], size=(8, 8))
    sign = rng.choice([-1.0, 1.0], size=(8, 8))
    h = 1e-3
    fd, pred = np.empty(8), np.empty(8)
    for t in range(8):
        Xp, Xm = X.copy(), X.copy()
        Xp[rows[t], cols[t]] += h * sign[t]
        Xm[rows[t], cols[t]] -= h * sign[t]
        sp, _ = oracle.silhouette(Xp, lab, spec.k)
        sm, _ = oracle.silhouette(Xm, lab, spec.k)
        fd[t] = np.sum(sp - sm) / X.shape[0] / (2 * h)
        pred[t] = np.sum(sign[t] * g[rows[t], cols[t]])
        print(f"  direction {t}: fd={fd[t]:.6e} grad={pred[t]:.6e}", flush=True)
    err = rel_l2(pred, fd)
    print(f"  FD rel_l2={err:.2e}", flush=True)
    assert err <= 1e-4
