"""The benchmark's command-line contract that holds without a GPU: one GPU only (a larger --gpus
exits with status 2 and says why, before anything touches a device), and the JSON field names of
the roofline and CPU-baseline objects."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_parse_defaults():
    sys.path.insert(0, ROOT)
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_cli", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    old = sys.argv
    try:
        sys.argv = ["bench.py"]
        args = bench.parse()
    finally:
        sys.argv = old
    assert args.gpus == 1 and args.workload == "blobs-50m-d128-k1000"
    assert args.metric == "sqeuclid" and args.form == "bf16"
    assert args.steps * 0.05 < 60  # the timed region stays well under a minute
    assert bench.PEAK["bf16"] == 2.5e15 and bench.PEAK["hbm"] == 8.0e12 and bench.PEAK["fp32"] == 157.3e12
