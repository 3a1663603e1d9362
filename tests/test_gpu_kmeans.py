"""K-means (Lloyd) step on the GPU against the FP64 oracle: labels where the two nearest means are
further apart than the distance bound, otherwise a label whose mean is within the bound of the
nearest; the inertia within the summed bounds; in-place updates, empty ids, repeated steps and
the error conventions."""

import numpy as np
import pytest
import torch

import oracle
from paper_2303_14102_amd import workloads as wl
from parity_helpers import dequantised, kmeans_dist_bound, storage

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_14102_amd import _lib
    _lib.load()  # fails loudly when the library is missing
    return torch.device("cuda:0")


def check_step(lab_gpu, inertia_gpu, Xh, lab_in, K, form, centre=True, products=3):
    """Xh: the values as stored (dequantised), widened here to binary64."""
    Xh = np.asarray(Xh, np.float64)
    lab_ref, inertia_ref, d1, d2 = oracle.kmeans_step(Xh, lab_in, K)
    bound = kmeans_dist_bound(form, centre, Xh, lab_in, K, products)
    clear = (d2 - d1) > 2 * bound
    same = lab_gpu == lab_ref
    assert np.all(same[clear]), f"{(~same[clear]).sum()} points with a clear nearest mean differ"
    # elsewhere: the GPU's mean must be within the bound of the nearest one
    idx = np.nonzero(~same)[0]
    if len(idx):
        ids = np.unique(lab_in)
        assert np.isin(lab_gpu[idx], ids).all(), "a point went to an empty cluster"
        mu = {int(k): Xh[lab_in == k].mean(axis=0) for k in ids}
        dg = np.array([((Xh[i] - mu[int(lab_gpu[i])]) ** 2).sum() for i in idx])
        assert np.all(dg <= d1[idx] + 2 * bound[idx])
    tol = 2 * bound.sum() + 1e-12 * inertia_ref
    assert abs(inertia_gpu - inertia_ref) <= tol, (inertia_gpu, inertia_ref, tol)
    return int((~same).sum()), int((~clear).sum())


CASES = [
    # (N, D, K, form, singletons, relabel, sigma, seed, products)
    (5_037, 40, 70, "f32", 2, 0.2, 2.0, 1, 0),
    (3_001, 128, 100, "bf16", 1, 0.3, 3.0, 2, 0),
    (2_000, 256, 40, "bf16", 0, 0.2, 1.5, 3, 0),
    (4_099, 16, 33, "fp8", 1, 0.2, 2.0, 4, 0),
    (1_500, 3, 5, "f32", 1, 0.3, 4.0, 5, 0),
    (1_500, 3, 5, "bf16", 0, 0.3, 4.0, 6, 0),
    (150_001, 64, 300, "bf16", 0, 0.1, 2.0, 7, 0),
    (140_333, 72, 257, "f32", 1, 0.1, 2.0, 8, 0),
    # two products on the exact x, folded centring
    (3_001, 128, 100, "bf16", 1, 0.3, 3.0, 9, 2),
    (2_000, 256, 40, "bf16", 0, 0.2, 1.5, 10, 2),
    (120_001, 128, 1000, "bf16", 1, 0.1, 2.0, 11, 2),
    (1_500, 3, 5, "bf16", 0, 0.3, 4.0, 12, 2),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c[0]}-D{c[1]}-K{c[2]}-{c[3]}-P{c[8]}")
def test_kmeans_step_parity(dev, case):
    from paper_2303_14102_amd import binding as sil
    n, d, k, form, single, relabel, sigma, seed, products = case
    b = wl.make_small(n, d, k, seed=seed, singletons=single, relabel=relabel, sigma=sigma)
    Kt = k + 2  # two unused ids
    Xd, sc, codes = storage(b.X.to(dev), form)
    print(f"[kmeans] N={n} D={d} K={Kt} form={form} products={products}", flush=True)
    lab_out, inertia = sil.kmeans_step(Xd, b.labels.to(dev), Kt, products=products, col_scale=sc,
                                       check_status=True)
    cs = None if sc is None else sc.cpu().numpy()
    Xh = dequantised(codes, cs)
    moved, near = check_step(lab_out.cpu().numpy(), inertia.item(), Xh, b.labels.numpy(), Kt, form,
                             products=products or 3)
    print(f"  moved-vs-oracle {moved}, near ties {near}, inertia {inertia.item():.6e}", flush=True)


def test_kmeans_in_place_and_uncentred(dev):
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(20_011, 40, 70, seed=9, singletons=2, relabel=0.2, sigma=2.0)
    X, lab = b.X.to(dev), b.labels.to(dev)
    out1, in1 = sil.kmeans_step(X, lab, 72, check_status=True)
    lab2 = lab.clone()
    out2, in2 = sil.kmeans_step(X, lab2, 72, labels_out=lab2, check_status=True)
    assert out2.data_ptr() == lab2.data_ptr()
    assert torch.equal(out1, lab2) and in1.item() == in2.item()
    out3, in3 = sil.kmeans_step(X, lab, 72, centre=False, check_status=True)
    check_step(out3.cpu().numpy(), in3.item(), b.X.numpy().astype(np.float64), b.labels.numpy(), 72,
               "f32", centre=False)


def test_kmeans_repeated_steps_do_not_increase_inertia(dev):
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(60_000, 32, 50, seed=10, relabel=0.5, sigma=3.0)
    X, lab = b.X.to(dev), b.labels.to(dev)
    ws = sil.new_workspace(60_000, 32, 50, "sqeuclid", X.dtype, 0, dev)
    prev = np.inf
    for it in range(6):
        lab, inertia = sil.kmeans_step(X, lab, 50, labels_out=lab, workspace=ws, check_status=True)
        v = inertia.item()
        print(f"[kmeans] step {it}: inertia {v:.8e}", flush=True)
        assert v <= prev * (1 + 1e-6)
        prev = v
    # the last step against the oracle from the same input labels
    lab_in = lab.clone()
    out, inertia = sil.kmeans_step(X, lab_in, 50, check_status=True)
    check_step(out.cpu().numpy(), inertia.item(), b.X.numpy().astype(np.float64), lab_in.cpu().numpy(),
               50, "f32")


def test_kmeans_single_nonempty_cluster(dev):
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(3_000, 8, 4, seed=11)
    lab = torch.full((3_000,), 2, dtype=torch.int32)
    out, inertia = sil.kmeans_step(b.X.to(dev), lab.to(dev), 4, check_status=True)
    assert torch.all(out.cpu() == 2)
    X = b.X.numpy().astype(np.float64)
    want = ((X - X.mean(axis=0)) ** 2).sum()
    assert abs(inertia.item() - want) <= 1e-5 * want


def test_kmeans_errors(dev):
    from paper_2303_14102_amd import _lib
    from paper_2303_14102_amd import binding as sil
    b = wl.make_small(2_000, 16, 5, seed=12)
    X = b.X.to(dev)
    bad = b.labels.clone()
    bad[7] = 5
    with pytest.raises(_lib.SilhouetteError) as e:
        sil.kmeans_step(X, bad.to(dev), 5, check_status=True)
    assert e.value.code == -3
    out, inertia = sil.kmeans_step(X, bad.to(dev), 5)
    torch.cuda.synchronize()
    assert torch.all(out == -1) and torch.isnan(inertia)
    Xb = X.to(torch.bfloat16)
    with pytest.raises(_lib.SilhouetteError) as e:  # one product is not offered
        sil.kmeans_step(Xb, b.labels.to(dev), 5, products=1)
    assert e.value.code == -1
    with pytest.raises(_lib.SilhouetteError) as e:  # two products need bf16 storage
        sil.kmeans_step(X, b.labels.to(dev), 5, products=2)
    assert e.value.code == -1
