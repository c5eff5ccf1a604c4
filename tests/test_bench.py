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
    t = bench.recorded_traffic("c2", 0)
    assert t is not None and t > 0
    assert bench.recorded_traffic("c2", 7) is None  # no such plan recorded
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0000000000000000")
    assert bench.recorded_traffic("c2", 0) is None
