"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic byte model and the
recorded-traffic lookup that is nulled when the kernel sources change."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_by_hand():
    # two 4 x 4 windows overlapping in a 2 x 2 corner, one minibatch of both:
    # 2 patterns x 16 px x 12 B + 28 touched px x 16 B + 16 probe px x 16 B
    pos = np.array([[0, 0], [2, 2]])
    A, U = bench.algorithmic_bytes_epoch(pos, np.array([0, 1]), 10, 4, 2)
    assert U == [28]
    assert A == 2 * 16 * 12 + 28 * 16 + 16 * 16
    # the same windows in two minibatches of one: each batch touches its own 16 px
    A1, U1 = bench.algorithmic_bytes_epoch(pos, np.array([1, 0]), 10, 4, 1)
    assert U1 == [16, 16]
    assert A1 == 2 * 16 * 12 + 32 * 16 + 2 * 16 * 16


def test_recorded_traffic_follows_the_sources(monkeypatch):
    import json
    rec = None
    with open(os.path.join(ROOT, "profiles", "patch_step_traffic.md")) as f:
        for line in f:
            if line.startswith("traffic_json: "):
                rec = json.loads(line[len("traffic_json: "):])
    assert rec is not None
    key = next(k for k in rec if "/plan" in k)
    wl, plan = key.split("/plan")
    # reported while the kernel sources match the digest recorded with the counters ...
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: rec["source"])
    t = bench.recorded_traffic(wl, int(plan))
    assert t is not None and t > 0
    assert bench.recorded_traffic(wl, 7) is None  # no such plan recorded
    # ... and null once they differ
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0000000000000000")
    assert bench.recorded_traffic(wl, int(plan)) is None


def test_time_to_target_spread_and_targets():
    assert bench.spread([None, None]) is None
    s = bench.spread([3.0, None, 1.0, 2.0])
    assert s == {"median": 2.0, "min": 1.0, "max": 3.0, "runs": 3}
    t = bench.load_targets("c2")
    assert "c2" in t and all(k == "c2" or k.startswith("c2/") for k in t)
    for v in t.values():
        assert abs(v["target"] - 1.01 * v["final"]) <= 1e-9 * v["target"]
        assert v["misfit"][-1] == v["final"] and len(v["misfit"]) == v["epochs"] + 1


def test_algorithmic_flops_per_pattern():
    # 64^2: two 2-D FFTs of 5 N log2 N flops (N = 4096, log2 N = 12) and 80 flops per pixel
    assert bench.algorithmic_flops_pattern(64) == 2 * 5 * 4096 * 12 + 80 * 4096
    assert abs(bench.VALU_PEAK_TFLOPS - 78.6432) < 1e-3
