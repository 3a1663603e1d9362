"""Persisted choices of the batched autotuner.

A JSON file maps a plan's signature to the launch configuration the tuner chose for it, so that a
later plan of the same shape applies that configuration instead of timing launches again.  The
signature is the GPU (architecture name and compute-unit count), the storage type, the plan's
flags and the multiset of its problems' (metric, D, K bucket, N bucket), where the K bucket is
ceil(log2 K) and the N bucket floor(log2 N): the order of the problems does not matter.

File format: {"format": 1, "entries": {key: {"config": {...}, "ms": float, "shape": str}}}.  A file
that cannot be read or has another format is treated as empty (and rewritten on the next store).
Stores replace the file atomically (a temporary file in the same folder, then rename)."""

from __future__ import annotations

import hashlib
import json
import math
import os
import tempfile
import warnings

FORMAT = 1


def k_bucket(K: int) -> int:
    return max(1, math.ceil(math.log2(K)))


def n_bucket(N: int) -> int:
    return max(0, int(N).bit_length() - 1)


def plan_key(arch: str, cus: int, dtype: str, flags: int, problems) -> tuple[str, str]:
    """(key, readable shape) for problems given as (metric, N, D, K) tuples."""
    items = sorted((str(m), int(D), k_bucket(int(K)), n_bucket(int(N))) for m, N, D, K in problems)
    counts = {}
    for it in items:
        counts[it] = counts.get(it, 0) + 1
    shape = ",".join(f"{m}/d{d}/k{k}/n{n}x{c}" for (m, d, k, n), c in counts.items())
    digest = hashlib.sha1(shape.encode()).hexdigest()[:16]
    return f"{arch}|cu{cus}|{dtype}|flags{flags}|p{len(items)}|{digest}", shape


class TuneCache:
    """The JSON cache at `path` (created on the first store)."""

    def __init__(self, path: str):
        self.path = os.path.abspath(path)
        self.entries = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    doc = json.load(f)
                if not isinstance(doc, dict) or doc.get("format") != FORMAT or not isinstance(
                        doc.get("entries"), dict):
                    raise ValueError("unknown format")
                self.entries = doc["entries"]
            except (OSError, ValueError) as e:
                warnings.warn(f"tune cache {self.path} ignored: {e}")
                self.entries = {}

    def get(self, key: str):
        e = self.entries.get(key)
        if not isinstance(e, dict) or not isinstance(e.get("config"), dict):
            return None
        cfg = dict(e["config"])
        # JSON object keys are strings: rows_per_item is keyed by GEMM depth
        cfg["rows_per_item"] = {int(k): int(v) for k, v in cfg.get("rows_per_item", {}).items()}
        return {"config": cfg, "ms": float(e.get("ms", 0.0))}

    def put(self, key: str, config: dict, ms: float, shape: str = "") -> None:
        self.entries[key] = {"config": config, "ms": float(ms), "shape": shape}
        folder = os.path.dirname(self.path)
        os.makedirs(folder, exist_ok=True)
        fd, tmp = tempfile.mkstemp(prefix=".tune-", suffix=".json", dir=folder)
        try:
            with os.fdopen(fd, "w") as f:
                json.dump({"format": FORMAT, "entries": self.entries}, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except BaseException:
            if os.path.exists(tmp):
                os.unlink(tmp)
            raise


__all__ = ["TuneCache", "plan_key", "k_bucket", "n_bucket", "FORMAT"]
