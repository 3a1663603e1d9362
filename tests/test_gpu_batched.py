"""Batched evaluation (k-sweep): every problem of a batch against the FP64 oracle and against the
single-problem entry point, for each launch configuration of the persistent kernel, the
autotuner's choice, hipGraph capture and replay, and per-problem error isolation.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_2303_14102_amd import workloads as wl
from parity_helpers import TOL_S_MEAN, bound_from_stats, per_point_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_14102_amd import _lib
    _lib.load()  # fails loudly when the library is missing
    return torch.device("cuda:0")


# (N, D, K, metric, singletons, seed): every GEMM depth class (16, 24, 32, 48, 64, 96, 128), ragged N,
# K from 2 to 300, both metrics, singleton clusters, rows fewer than one block
MIXED = [
    (3_001, 3, 5, "sqeuclid", 1, 31),
    (1_500, 15, 2, "cosine", 0, 32),
    (4_099, 16, 33, "sqeuclid", 1, 33),
    (2_000, 23, 64, "cosine", 2, 34),
    (5_037, 32, 70, "sqeuclid", 0, 35),
    (900, 39, 7, "sqeuclid", 1, 36),
    (2_500, 40, 100, "cosine", 0, 37),
    (3_333, 64, 130, "sqeuclid", 1, 38),
    (77, 71, 3, "sqeuclid", 0, 39),
    (2_222, 100, 250, "cosine", 1, 40),
    (4_000, 128, 300, "sqeuclid", 2, 41),
    (1_000, 128, 2, "cosine", 0, 42),
]


def make_problems(dev):
    probs, refs = [], []
    for n, d, k, metric, single, seed in MIXED:
        b = wl.make_small(n, d, k, seed=seed, singletons=single)
        probs.append((b.X.to(dev), b.labels.to(dev), k, metric))
        refs.append((b.X.numpy(), b.labels.numpy(), k, metric))
    return probs, refs


@pytest.fixture(scope="module")
def mixed(dev):
    probs, refs = make_problems(dev)
    expect = []
    for X, lab, k, metric in refs:
        s_ref, S_ref, a, b, _ = oracle.silhouette(X, lab, k, metric, details=True)
        bound = per_point_bound("f32", 0, metric, True, X, lab, k, a, b)
        expect.append((s_ref, S_ref, bound))
    return probs, refs, expect


def check_against_oracle(batch, expect, tag):
    torch.cuda.synchronize()
    assert batch.status() == [0] * len(expect), tag
    S = batch.S.cpu().numpy()
    for i, (s_ref, S_ref, bound) in enumerate(expect):
        s = batch.s[i].cpu().numpy().astype(np.float64)
        ds = np.abs(s - s_ref)
        assert np.all(ds <= bound), f"{tag} problem {i} ({MIXED[i]}): point {int((ds / bound).argmax())}"
        assert abs(S[i] - S_ref) <= TOL_S_MEAN["f32"], f"{tag} problem {i}: S {S[i]} vs {S_ref}"


CONFIGS = [
    dict(grid=512, grab=1, order="cost"),
    dict(grid=256, grab=4, order="problem", rows_per_item={16: 256, 24: 256, 32: 256}),
    dict(grid=768, grab=2, order="cost", rows_per_item={24: 256}),
    dict(grid=7, grab=64, order="problem", rows_per_item={16: 256, 32: 256}),
]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: f"g{c['grid']}-x{c['grab']}-{c['order']}")
def test_batched_matches_oracle(dev, mixed, cfg):
    from paper_2303_14102_amd import BatchedSilhouette
    probs, refs, expect = mixed
    print(f"[batched] {len(probs)} problems, config {cfg}", flush=True)
    batch = BatchedSilhouette(probs)
    batch.set_config(**cfg)
    batch.run()
    check_against_oracle(batch, expect, str(cfg))
    batch.run()  # a second run on the same workspace (no upload) gives the same result
    check_against_oracle(batch, expect, str(cfg) + " again")
    batch.close()


def test_batched_equals_single_problem_calls(dev, mixed):
    from paper_2303_14102_amd import BatchedSilhouette
    from paper_2303_14102_amd import binding as sil
    probs, _, _ = mixed
    batch = BatchedSilhouette(probs)
    batch.run()
    torch.cuda.synchronize()
    for i, (X, lab, k, metric) in enumerate(probs):
        s1, S1 = sil.silhouette(X, lab, k, metric, check_status=True)
        # same kernels, same arithmetic per point; the statistics' FP64 sums may differ in the
        # order of rows within a cluster
        assert abs(batch.S[i].item() - S1.item()) <= 1e-12
        np.testing.assert_allclose(batch.s[i].cpu().numpy(), s1.cpu().numpy(), rtol=0, atol=1e-6)


def test_batched_offset_labels(dev, mixed):
    # labels that start 4 bytes past an aligned address: the histogram and the staged scatter take
    # their 4-byte label loads for those problems, the 16-byte ones for the others
    from paper_2303_14102_amd import BatchedSilhouette
    probs, _, expect = mixed
    shifted = []
    for i, (X, lab, k, metric) in enumerate(probs):
        if i % 2 == 0:
            buf = torch.empty(lab.numel() + 1, dtype=torch.int32, device=dev)
            buf[1:] = lab
            lab = buf[1:]
            assert lab.data_ptr() % 16 == 4
        shifted.append((X, lab, k, metric))
    batch = BatchedSilhouette(shifted)
    batch.run()
    check_against_oracle(batch, expect, "offset labels")
    batch.close()


def test_autotuner_choice(dev, mixed):
    from paper_2303_14102_amd import BatchedSilhouette
    probs, _, expect = mixed
    batch = BatchedSilhouette(probs)
    ms = batch.tune()
    cfg = batch.config()
    print(f"[batched] tuned: {ms:.3f} ms, {cfg}", flush=True)
    assert ms > 0 and cfg["grid"] >= 1 and cfg["grab"] in (1, 2, 4)
    check_against_oracle(batch, expect, f"tuned {cfg}")
    batch.run()
    check_against_oracle(batch, expect, "tuned, run")


def test_tune_cache(dev, mixed, tmp_path):
    # the first plan is tuned and its choice stored; a second plan of the same shape takes it from
    # the cache without timing launches, and its results still match the oracle
    from paper_2303_14102_amd import BatchedSilhouette
    probs, _, expect = mixed
    path = str(tmp_path / "tune.json")
    first = BatchedSilhouette(probs)
    ms = first.tune(cache=path)
    assert not first.tuned_from_cache and ms > 0
    cfg = first.config()
    first.close()
    second = BatchedSilhouette(probs)
    assert second.tune(cache=path) == ms
    assert second.tuned_from_cache and second.config() == cfg
    check_against_oracle(second, expect, f"cached {cfg}")
    second.close()


def test_graph_capture_and_replay(dev, mixed):
    from paper_2303_14102_amd import BatchedSilhouette
    from paper_2303_14102_amd import binding as sil
    probs, _, expect = mixed
    batch = BatchedSilhouette(probs)
    batch.run()
    torch.cuda.synchronize()
    S_eager = batch.S.clone()
    s_eager = [s.clone() for s in batch.s]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    batch.capture(side)
    side.synchronize()
    for rep in range(4):
        batch.S.fill_(float("nan"))
        for s in batch.s:
            s.fill_(float("nan"))
        torch.cuda.synchronize()
        batch.replay(side)
        side.synchronize()
        print(f"[batched] replay {rep}", flush=True)
        assert torch.allclose(batch.S, S_eager, rtol=0, atol=1e-12), rep
        for i in range(len(probs)):
            assert torch.allclose(batch.s[i], s_eager[i], rtol=0, atol=1e-6), (rep, i)
        # the program's own eager work between replays
        X, lab, k, metric = probs[rep % len(probs)]
        sil.silhouette(X, lab, k, metric, check_status=True)
        (torch.randn(256, 256, device=dev) @ torch.randn(256, 256, device=dev)).sum().item()
    check_against_oracle(batch, expect, "after replays")


def test_batched_euclid_approx(dev, mixed):
    # the approximate Euclidean flag applies to the squared Euclidean problems of the batch; the
    # cosine problems ignore it
    from paper_2303_14102_amd import BatchedSilhouette
    probs, refs, _ = mixed
    batch = BatchedSilhouette(probs, euclid_approx=True)
    batch.run()
    torch.cuda.synchronize()
    assert batch.status() == [0] * len(probs)
    S = batch.S.cpu().numpy()
    for i, (X, lab, k, metric) in enumerate(refs):
        m = "euclid_approx" if metric == "sqeuclid" else metric
        s_ref, S_ref, a, b, _ = oracle.silhouette(X, lab, k, m, details=True)
        bound = per_point_bound("f32", 0, m, True, X, lab, k, a, b)
        ds = np.abs(batch.s[i].cpu().numpy().astype(np.float64) - s_ref)
        assert np.all(ds <= bound), f"problem {i} ({MIXED[i]}): point {int((ds / bound).argmax())}"
        assert abs(S[i] - S_ref) <= TOL_S_MEAN["f32"], f"problem {i}: S {S[i]} vs {S_ref}"
    batch.close()


# Problems that share X (labelings of one data set) run as a group: one pass over the rows for
# all its members.  Two data sets (D = 32: depth 32, where two row blocks per wave are possible;
# D = 100: depth 128, ragged N), several labelings each (K from 2 to 300, singletons, a random
# labeling), a standalone problem between them, and a cosine labeling of the first data set
# (another metric: its own group).
def make_group_problems(dev):
    rng = np.random.default_rng(64)
    a = wl.make_small(5_003, 32, 40, seed=61, singletons=1)
    b = wl.make_small(3_001, 100, 12, seed=62)
    c = wl.make_small(2_000, 16, 9, seed=63)
    la, lb = a.labels.numpy(), b.labels.numpy()
    labs = [
        ("a", la, 40, "sqeuclid"),
        ("a", wl.ksweep_labels(la, 40, 7, 0.05, rng), 7, "sqeuclid"),
        ("c", c.labels.numpy(), 9, "sqeuclid"),
        ("a", rng.integers(0, 300, len(la)).astype(np.int32), 300, "sqeuclid"),
        ("a", la, 40, "cosine"),
        ("b", lb, 12, "cosine"),
        ("b", wl.ksweep_labels(lb, 12, 3, 0.02, rng), 3, "cosine"),
        ("b", rng.integers(0, 2, len(lb)).astype(np.int32), 2, "cosine"),
    ]
    X = {"a": a.X, "b": b.X, "c": c.X}
    Xd = {k: v.to(dev) for k, v in X.items()}
    probs, refs = [], []
    for name, lab, k, metric in labs:
        probs.append((Xd[name], torch.from_numpy(np.ascontiguousarray(lab)).to(dev), k, metric))
        refs.append((X[name].numpy(), lab, k, metric))
    return probs, refs


@pytest.fixture(scope="module")
def grouped(dev):
    probs, refs = make_group_problems(dev)
    expect = []
    for X, lab, k, metric in refs:
        s_ref, S_ref, a, b, _ = oracle.silhouette(X, lab, k, metric, details=True)
        bound = per_point_bound("f32", 0, metric, True, X, lab, k, a, b)
        expect.append((s_ref, S_ref, bound))
    return probs, refs, expect


@pytest.mark.parametrize("share", [True, False])
@pytest.mark.parametrize("cfg", [dict(grid=512, grab=1, order="cost"),
                                 dict(grid=7, grab=3, order="problem", rows_per_item={32: 256})],
                         ids=["g512", "g7-rows256"])
def test_shared_rows_groups(dev, grouped, cfg, share):
    from paper_2303_14102_amd import BatchedSilhouette
    probs, _, expect = grouped
    print(f"[batched-groups] share_x={share} {cfg}", flush=True)
    batch = BatchedSilhouette(probs)
    batch.set_config(**cfg, share_x=share)
    assert batch.config()["share_x"] == share
    batch.run()
    torch.cuda.synchronize()
    assert batch.status() == [0] * len(probs)
    S = batch.S.cpu().numpy()
    for i, (s_ref, S_ref, bound) in enumerate(expect):
        ds = np.abs(batch.s[i].cpu().numpy().astype(np.float64) - s_ref)
        assert np.all(ds <= bound), f"problem {i}: point {int((ds / bound).argmax())}"
        assert abs(S[i] - S_ref) <= TOL_S_MEAN["f32"], f"problem {i}: S {S[i]} vs {S_ref}"
    batch.close()


def test_shared_rows_match_separate_passes(dev, grouped):
    # the same per-row arithmetic either way, but for two roundings: a member's tables are
    # centred with the leader's vector (its FP64 sum runs over other clusters in another order,
    # so a table entry can round to the neighbouring fp32 value), and a member's cosine a-path
    # starts from the stored z = x / |x| where the prologue may fuse that product into its first
    # difference (measured: squared Euclidean identical, cosine members |dS| <= 8.4e-10)
    from paper_2303_14102_amd import BatchedSilhouette
    probs, _, _ = grouped
    out = []
    for share in (True, False):
        batch = BatchedSilhouette(probs)
        batch.set_config(grid=512, share_x=share)
        batch.run()
        torch.cuda.synchronize()
        out.append((batch.S.cpu().numpy(), [s.cpu().numpy() for s in batch.s]))
        batch.close()
    (S1, s1), (S0, s0) = out
    dS = np.abs(S1 - S0)
    ds = [float(np.abs(a.astype(np.float64) - b).max()) for a, b in zip(s1, s0)]
    print(f"  |dS| per problem {dS}, max |ds| {ds}", flush=True)
    assert np.all(dS <= 1e-9)
    assert max(ds) <= 1e-6


def test_errors_inside_a_group_are_isolated(dev):
    # three labelings of one data set: the leader and the last member carry a label outside
    # [0, K); the middle member, which takes the leader's centring vector, is still exact
    from paper_2303_14102_amd import BatchedSilhouette
    d = wl.make_small(3_000, 24, 8, seed=71)
    X = d.X.to(dev)
    lab = d.labels.numpy()
    bad0, bad2 = lab.copy(), lab.copy()
    bad0[5] = 8
    bad2[2_999] = -2
    probs = [(X, torch.from_numpy(l).to(dev), 8, "sqeuclid") for l in (bad0, lab, bad2)]
    batch = BatchedSilhouette(probs)
    batch.run()
    torch.cuda.synchronize()
    assert batch.status() == [-3, 0, -3]  # SIL_E_LABEL
    S = batch.S.cpu().numpy()
    assert np.isnan(S[0]) and np.isnan(S[2])
    s_ref, S_ref, a, b, _ = oracle.silhouette(d.X.numpy(), lab, 8, details=True)
    bound = per_point_bound("f32", 0, "sqeuclid", True, d.X.numpy(), lab, 8, a, b)
    ds = np.abs(batch.s[1].cpu().numpy().astype(np.float64) - s_ref)
    assert np.all(ds <= bound) and abs(S[1] - S_ref) <= TOL_S_MEAN["f32"]
    batch.close()


def test_error_in_one_problem_is_isolated(dev):
    from paper_2303_14102_amd import BatchedSilhouette
    good = wl.make_small(2_000, 16, 10, seed=50)
    bad = wl.make_small(1_000, 32, 6, seed=51)
    lab_bad = bad.labels.clone()
    lab_bad[17] = 6  # outside [0, K)
    zero = wl.make_small(1_500, 8, 4, seed=52)
    Xz = zero.X.clone()
    Xz[3] = 0.0      # a zero row under the cosine distance
    probs = [(good.X.to(dev), good.labels.to(dev), 10, "sqeuclid"),
             (bad.X.to(dev), lab_bad.to(dev), 6, "sqeuclid"),
             (Xz.to(dev), zero.labels.to(dev), 4, "cosine"),
             (good.X.to(dev), good.labels.to(dev), 10, "cosine")]
    batch = BatchedSilhouette(probs)
    batch.run()
    st = batch.status()
    assert st == [0, -3, -5, 0], st
    S = batch.S.cpu().numpy()
    assert math.isnan(S[1]) and math.isnan(S[2])
    assert torch.isnan(batch.s[1]).all() and torch.isnan(batch.s[2]).all()
    for i, metric in ((0, "sqeuclid"), (3, "cosine")):
        _, S_ref = oracle.silhouette(good.X.numpy(), good.labels.numpy(), 10, metric)
        assert abs(S[i] - S_ref) <= 1e-6


def test_ksweep_workload_sampled(dev):
    # the batched k-sweep workload at its full size: 32 data sets of 1e4..2e6 points in 16..128
    # dimensions, 8 labelings each (K from 2 to 256); sampled points of every problem against
    # the oracle's linear form (FP64 statistics of all rows), S against the mean of its s_i
    from paper_2303_14102_amd import BatchedSilhouette
    print("[ksweep] generating", flush=True)
    data = wl.make_ksweep(device=dev)
    probs = [(ds.X, lab, k, "sqeuclid") for ds in data for k, lab in ds.labelings]
    print(f"[ksweep] {len(probs)} problems, {sum(p[0].shape[0] for p in probs)} points", flush=True)
    batch = BatchedSilhouette(probs)
    ms = batch.tune()
    print(f"[ksweep] tuned {ms:.2f} ms {batch.config()}", flush=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    batch.capture(side)
    batch.replay(side)
    side.synchronize()
    assert all(v == 0 for v in batch.status())
    S = batch.S.cpu().numpy()
    rng = np.random.default_rng(11)
    worst = 0.0
    for d, ds in enumerate(data):
        Xh = ds.X.cpu().numpy()
        for j, (k, lab) in enumerate(ds.labelings):
            i = d * len(ds.labelings) + j
            lab_h = lab.cpu().numpy()
            s = batch.s[i].cpu().numpy().astype(np.float64)
            assert abs(S[i] - s.sum() / len(s)) <= 1e-12
            if j % 4:  # oracle on every fourth labeling keeps the test within its time
                continue
            stats = oracle.cluster_stats(Xh, lab_h, k, "sqeuclid")
            idx = rng.choice(len(s), size=64, replace=False)
            s_lin, a, b, _ = oracle.scores_at(Xh, lab_h, k, idx, stats, "sqeuclid")
            bound = bound_from_stats("f32", 0, "sqeuclid", True, Xh[idx], stats, a, b)
            ds_ = np.abs(s[idx] - s_lin)
            worst = max(worst, float((ds_ / bound).max()))
            assert np.all(ds_ <= bound), f"problem {i} (data set {d}, K={k})"
    print(f"[ksweep] worst |ds|/bound {worst:.3f}", flush=True)
