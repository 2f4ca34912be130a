"""Host-side logic that needs no GPU: the benchmark's one-GPU contract, its counter-summary
reader, and the binding's argument checks that run before any library call."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    import bench
    traffic, note = bench.counter_traffic(bench.KERNEL_SOURCES)
    if traffic is not None:
        assert traffic > 7e8 and "calibrated" in note
    # a source list whose hash differs from the summary's gives no traffic figure
    t2, note2 = bench.counter_traffic(["bench.py"])
    assert t2 is None and "changed" in note2


def test_qam_gray_inputs():
    """Square Gray QAM of the input generator: unit energy per 2D, a permutation of labels,
    and neighbours on the grid differ in exactly one label bit."""
    import numpy as np
    import synth
    for M in (4, 16, 64, 256):
        X, labels = synth.qam_gray(M)
        assert abs(float((X.astype(np.float64) ** 2).sum(1).mean()) - 1.0) < 1e-6
        assert sorted(labels.tolist()) == list(range(M))
        L = int(round(M ** 0.5))
        for i in range(L):
            for q in range(L):
                j = i * L + q
                for jj in ([(i + 1) * L + q] if i + 1 < L else []) + ([i * L + q + 1] if q + 1 < L else []):
                    assert bin(int(labels[j]) ^ int(labels[jj])).count("1") == 1
