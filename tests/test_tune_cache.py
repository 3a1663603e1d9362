"""Host logic of the batched tuner's persisted cache (paper_2303_14102_amd/tune_cache.py)."""

import json
import os
import warnings

from paper_2303_14102_amd.tune_cache import TuneCache, k_bucket, n_bucket, plan_key

PROBS = [("sqeuclid", 10_000, 16, 5), ("cosine", 2_000_000, 128, 256), ("sqeuclid", 77, 3, 2)]
CFG = {"grid": 512, "grab": 2, "order": "problem", "rows_per_item": {16: 256, 24: 128, 32: 128}}


def test_buckets():
    assert [k_bucket(k) for k in (2, 3, 4, 5, 8, 9, 256, 257)] == [1, 2, 2, 3, 3, 4, 8, 9]
    assert [n_bucket(n) for n in (1, 2, 3, 4, 1023, 1024)] == [0, 1, 1, 2, 9, 10]


def test_key_ignores_order_and_separates_shapes():
    k0, shape = plan_key("gfx950", 256, "f32", 0, PROBS)
    assert plan_key("gfx950", 256, "f32", 0, PROBS[::-1])[0] == k0
    assert "sqeuclid/d16/k3/n13x1" in shape
    # same buckets: same key (K 5 -> 6, N 10,000 -> 12,000)
    assert plan_key("gfx950", 256, "f32", 0, [("sqeuclid", 12_000, 16, 6)] + PROBS[1:])[0] == k0
    others = [
        plan_key("gfx942", 256, "f32", 0, PROBS),
        plan_key("gfx950", 304, "f32", 0, PROBS),
        plan_key("gfx950", 256, "f32", 1, PROBS),
        plan_key("gfx950", 256, "f32", 0, [("sqeuclid", 10_000, 16, 9)] + PROBS[1:]),
        plan_key("gfx950", 256, "f32", 0, [("sqeuclid", 10_000, 17, 5)] + PROBS[1:]),
        plan_key("gfx950", 256, "f32", 0, [("cosine", 10_000, 16, 5)] + PROBS[1:]),
        plan_key("gfx950", 256, "f32", 0, [("sqeuclid", 20_000, 16, 5)] + PROBS[1:]),
        plan_key("gfx950", 256, "f32", 0, PROBS + PROBS[:1]),
    ]
    assert len({k for k, _ in others} | {k0}) == len(others) + 1


def test_round_trip(tmp_path):
    path = os.path.join(tmp_path, "sub", "tune.json")
    key, shape = plan_key("gfx950", 256, "f32", 0, PROBS)
    c = TuneCache(path)
    assert c.get(key) is None
    c.put(key, CFG, 12.5, shape)
    got = TuneCache(path).get(key)
    assert got == {"config": CFG, "ms": 12.5}
    assert isinstance(next(iter(got["config"]["rows_per_item"])), int)
    doc = json.load(open(path))
    assert doc["format"] == 1 and doc["entries"][key]["shape"] == shape
    # a second entry keeps the first; no temporary files are left behind
    k2, s2 = plan_key("gfx950", 256, "f32", 1, PROBS)
    TuneCache(path).put(k2, {**CFG, "grid": 7}, 3.0, s2)
    c3 = TuneCache(path)
    assert c3.get(key)["config"]["grid"] == 512 and c3.get(k2)["config"]["grid"] == 7
    assert sorted(os.listdir(os.path.dirname(path))) == ["tune.json"]


def test_unreadable_files_are_ignored(tmp_path):
    key, _ = plan_key("gfx950", 256, "f32", 0, PROBS)
    for text in ("{not json", json.dumps({"format": 99, "entries": {}}), json.dumps([1, 2])):
        path = os.path.join(tmp_path, "bad.json")
        with open(path, "w") as f:
            f.write(text)
        with warnings.catch_warnings(record=True) as w:
            warnings.simplefilter("always")
            c = TuneCache(path)
        assert c.entries == {} and any("ignored" in str(x.message) for x in w)
        c.put(key, CFG, 1.0)  # rewritten in the current format
        assert TuneCache(path).get(key)["config"] == CFG
