"""Seeded synthetic clustering workloads (Gaussian blobs) shared by the HIP path and the oracle.

This module only draws inputs: cluster centres, cluster sizes, labels and points, plus the
storage formats the precision forms read (bf16 codes, fp8 e4m3 codes with a per-column
power-of-two scale).  It holds none of the Silhouette arithmetic (cluster statistics, mean
distances, a_i/b_i/s_i); that lives in the HIP kernels on one side and in the oracle on the
other, and neither imports the other.

The paper measures on a proprietary 129-feature dataset (Section IV), which is not available;
seeded Gaussian blobs with the sizes, dimensionalities, cluster counts and size distributions of
the named workloads stand in for it.

Recipe (all structure on the host with numpy's PCG64, the noise with torch's generator on the
target device so that 25 GB inputs are drawn where they live):
  1. centres c_k ~ U[lo, hi]^D;
  2. cluster sizes: Dirichlet(1) weights or Zipf(s) weights, largest-remainder rounding with a
     minimum of 2 points per cluster, optionally plus singleton clusters (size 1);
  3. true labels = each cluster id repeated by its size, then a seeded permutation of the rows;
  4. x_i = c_{true label} + sigma * N(0, I), rounded to fp32;
  5. relabel noise: exactly round(p * N) rows (never from or into a singleton cluster) get a
     label drawn uniformly from the other non-singleton clusters.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

# --------------------------------------------------------------------------------------------
# named workloads


@dataclasses.dataclass(frozen=True)
class BlobSpec:
    name: str
    n: int
    d: int
    k: int
    sigma: float
    sizes: str = "dirichlet"  # "dirichlet" | "zipf"
    zipf_s: float = 1.1
    singletons: int = 0
    relabel: float = 0.05
    seed: int = 0
    centre_lo: float = -10.0
    centre_hi: float = 10.0


WORKLOADS = {
    # small plain-method case, both metrics
    "blobs-10k-d8-k4": BlobSpec("blobs-10k-d8-k4", 10_000, 8, 4, 1.0, "dirichlet", relabel=0.05, seed=0),
    # plain fp32 at scale: Zipf(1.1) sizes over 97 clusters plus 3 singletons, 10% relabel
    "blobs-10m-d64-k100": BlobSpec("blobs-10m-d64-k100", 10_000_000, 64, 100, 2.0, "zipf", 1.1,
                                   singletons=3, relabel=0.10, seed=1),
    # precision-form workload (bf16 / fp8 storage compared with fp32)
    "blobs-50m-d128-k1000": BlobSpec("blobs-50m-d128-k1000", 50_000_000, 128, 1000, 1.0, "dirichlet",
                                     relabel=0.05, seed=2),
    # differentiation workload
    "blobs-1m-d256-k64": BlobSpec("blobs-1m-d256-k64", 1_000_000, 256, 64, 1.5, "dirichlet",
                                  relabel=0.05, seed=4),
}


def scaled(spec: BlobSpec, n: int, name: Optional[str] = None) -> BlobSpec:
    """Same recipe with a different point count (for tests that need a bounded size)."""
    return dataclasses.replace(spec, n=n, name=name or f"{spec.name}@n{n}")


# --------------------------------------------------------------------------------------------
# sizes


def _largest_remainder(weights: np.ndarray, total: int, minimum: int) -> np.ndarray:
    k = len(weights)
    if total < minimum * k:
        raise ValueError(f"cannot give {k} clusters at least {minimum} of {total} points")
    free = total - minimum * k
    w = np.asarray(weights, dtype=np.float64)
    w = w / w.sum()
    raw = w * free
    base = np.floor(raw).astype(np.int64)
    short = free - int(base.sum())
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:short]] += 1
    return base + minimum


def cluster_sizes(spec: BlobSpec, rng: np.random.Generator) -> np.ndarray:
    """Sizes per cluster id (after a seeded shuffle of ids, so singletons are not last)."""
    k_main = spec.k - spec.singletons
    n_main = spec.n - spec.singletons
    if spec.sizes == "dirichlet":
        w = rng.dirichlet(np.ones(k_main))
    elif spec.sizes == "zipf":
        w = np.arange(1, k_main + 1, dtype=np.float64) ** (-spec.zipf_s)
    else:
        raise ValueError(spec.sizes)
    sizes = np.concatenate([_largest_remainder(w, n_main, 2), np.ones(spec.singletons, np.int64)])
    return sizes[rng.permutation(spec.k)]


# --------------------------------------------------------------------------------------------
# points and labels


@dataclasses.dataclass
class Blobs:
    spec: BlobSpec
    X: torch.Tensor        # [N, D] float32 on `device`
    labels: torch.Tensor   # [N] int32 on `device` (observed labels, with relabel noise)
    sizes: np.ndarray      # true cluster sizes


def make_labels(spec: BlobSpec) -> tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """(true_labels, observed_labels, sizes, centres) drawn on the host."""
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    centres = rng.uniform(spec.centre_lo, spec.centre_hi, size=(spec.k, spec.d))
    sizes = cluster_sizes(spec, rng)
    true = np.repeat(np.arange(spec.k, dtype=np.int32), sizes)
    true = true[rng.permutation(spec.n)]
    observed = true.copy()
    m = int(round(spec.relabel * spec.n))
    if m:
        big = sizes >= 2
        movable = np.flatnonzero(big[true])
        rows = rng.choice(movable, size=m, replace=False)
        targets = np.flatnonzero(big).astype(np.int32)
        # uniform over the other non-singleton clusters: draw from len-1 slots, skip own slot
        pos_of = np.full(spec.k, -1, np.int64)
        pos_of[targets] = np.arange(len(targets))
        own = pos_of[true[rows]]
        r = rng.integers(0, len(targets) - 1, size=m)
        r = r + (r >= own)
        observed[rows] = targets[r]
    return true, observed, sizes, centres


def make_blobs(spec: BlobSpec, device: str | torch.device = "cpu", chunk_rows: int = 1 << 22) -> Blobs:
    true, observed, sizes, centres = make_labels(spec)
    device = torch.device(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(1_000_003 * spec.seed + 17)
    c = torch.from_numpy(centres.astype(np.float32)).to(device)
    X = torch.empty((spec.n, spec.d), dtype=torch.float32, device=device)
    lab_true = torch.from_numpy(true).to(device)
    for r0 in range(0, spec.n, chunk_rows):
        r1 = min(spec.n, r0 + chunk_rows)
        noise = torch.randn((r1 - r0, spec.d), generator=gen, device=device, dtype=torch.float32)
        X[r0:r1] = c[lab_true[r0:r1].long()] + spec.sigma * noise
        del noise
    labels = torch.from_numpy(observed).to(device)
    return Blobs(spec, X, labels, sizes)


def make_small(n: int, d: int, k: int, seed: int, sigma: float = 1.0, relabel: float = 0.05,
               singletons: int = 0, device: str = "cpu") -> Blobs:
    spec = BlobSpec(f"blobs-{n}-d{d}-k{k}-s{seed}", n, d, k, sigma, "dirichlet", relabel=relabel,
                    singletons=singletons, seed=seed)
    return make_blobs(spec, device)


# --------------------------------------------------------------------------------------------
# storage formats for the precision forms


def to_bf16(X: torch.Tensor) -> torch.Tensor:
    """fp32 -> bf16, round to nearest even (torch's conversion)."""
    return X.to(torch.bfloat16)


FP8_E4M3_MAX = 448.0


def to_fp8_e4m3(X: torch.Tensor, chunk_rows: int = 1 << 22) -> tuple[torch.Tensor, torch.Tensor]:
    """fp32 -> (fp8 e4m3fn codes [N,D], fp32 per-column scale [D]).

    The scale of column l is the power of two 2^ceil(log2(amax_l / 448)), so that code * scale
    is exact in fp32 and no code saturates.  Codes are round-to-nearest-even (torch).
    """
    amax = torch.zeros(X.shape[1], dtype=torch.float32, device=X.device)
    for r0 in range(0, X.shape[0], chunk_rows):
        amax = torch.maximum(amax, X[r0:r0 + chunk_rows].abs().amax(dim=0))
    amax = torch.clamp(amax, min=torch.finfo(torch.float32).tiny)
    scale = torch.exp2(torch.ceil(torch.log2(amax / FP8_E4M3_MAX)))
    q = torch.empty(X.shape, dtype=torch.float8_e4m3fn, device=X.device)
    for r0 in range(0, X.shape[0], chunk_rows):
        q[r0:r0 + chunk_rows] = (X[r0:r0 + chunk_rows] / scale).to(torch.float8_e4m3fn)
    return q, scale


def host_codes(X: torch.Tensor) -> np.ndarray:
    """Raw storage of X on the host as numpy: float32, uint16 bf16 bits or uint8 fp8 codes."""
    if X.dtype == torch.float32:
        return X.detach().cpu().numpy()
    if X.dtype == torch.bfloat16:
        return X.detach().cpu().view(torch.int16).numpy().view(np.uint16)
    if X.dtype == torch.float8_e4m3fn:
        return X.detach().cpu().view(torch.uint8).numpy()
    raise TypeError(X.dtype)


# --------------------------------------------------------------------------------------------
# k-sweep: several labelings of each of several data sets


@dataclasses.dataclass
class SweepDataset:
    X: torch.Tensor                 # [N, D] float32 on the device
    blob: np.ndarray                # true blob id of every row (host)
    labelings: list                 # [(K, labels int32 [N] on the device)]


def ksweep_labels(blob: np.ndarray, n_blobs: int, k: int, relabel: float,
                  rng: np.random.Generator) -> np.ndarray:
    """Merge blobs into k clusters (blob b -> floor(b k / n_blobs)), then move exactly
    round(relabel N) rows to a cluster drawn uniformly from the other k - 1."""
    lab = (blob.astype(np.int64) * k // n_blobs).astype(np.int32)
    m = int(round(relabel * len(blob)))
    if m:
        rows = rng.choice(len(blob), size=m, replace=False)
        r = rng.integers(0, k - 1, size=m).astype(np.int32)
        lab[rows] = r + (r >= lab[rows])
    return lab


def make_ksweep(n_datasets: int = 32, labelings: int = 8, n_lo: int = 10_000, n_hi: int = 2_000_000,
                dims=(16, 32, 64, 128), n_blobs: int = 256, k_lo: int = 2, k_hi: int = 256,
                sigma: float = 1.0, relabel: float = 0.05, seed0: int = 1000,
                device: str | torch.device = "cpu") -> list:
    """The batched k-sweep workload: data set d (seed seed0 + d) has N ~ U_int[n_lo, n_hi] points
    in D ~ U(dims) dimensions drawn as n_blobs Gaussian blobs (centres U[-10, 10]^D, Dirichlet(1)
    sizes, sigma); each of its `labelings` labelings has K log-uniform in [k_lo, k_hi] (integer)
    and merges the blobs into K clusters, with relabel noise."""
    out = []
    for d in range(n_datasets):
        rng = np.random.Generator(np.random.PCG64(seed0 + d))
        n = int(rng.integers(n_lo, n_hi + 1))
        dim = int(rng.choice(np.asarray(dims)))
        spec = BlobSpec(f"ksweep-{d}", n, dim, n_blobs, sigma, "dirichlet", relabel=0.0, seed=seed0 + d)
        b = make_blobs(spec, device)
        blob = b.labels.cpu().numpy()
        labs = []
        for _ in range(labelings):
            k = int(np.clip(np.round(np.exp(rng.uniform(np.log(k_lo), np.log(k_hi)))), k_lo, k_hi))
            lab = ksweep_labels(blob, n_blobs, k, relabel, rng)
            labs.append((k, torch.from_numpy(lab).to(device)))
        out.append(SweepDataset(b.X, blob, labs))
    return out


def expected_size_bytes(spec: BlobSpec, bytes_per_elem: int) -> int:
    return spec.n * spec.d * bytes_per_elem + 4 * spec.n


def fits(spec: BlobSpec, free_bytes: int, bytes_per_elem: int = 4) -> bool:
    return expected_size_bytes(spec, bytes_per_elem) * 2 < free_bytes


__all__ = ["BlobSpec", "WORKLOADS", "Blobs", "make_blobs", "make_small", "make_labels", "scaled",
           "cluster_sizes", "to_bf16", "to_fp8_e4m3", "host_codes", "FP8_E4M3_MAX", "SweepDataset",
           "ksweep_labels", "make_ksweep"]
