"""Host-side statistics of the serving bench: queue depth and latency
percentiles against their definitions, counted by brute force."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_queue_depth_worked_example():
    arr = [0.0, 1.0, 2.0, 3.0]
    done = [0.5, 2.5, 2.6, 3.1]
    st = bench.serving_stats(arr, done)
    # in the system at each arrival: {0}, {1}, {1, 2}, {3}
    assert st["max_queue_depth"] == 2
    assert st["mean_queue_depth"] == 5 / 4
    assert np.isclose(st["p50_latency_ms"], np.percentile([500.0, 1500.0, 600.0, 100.0], 50))


def test_queue_depth_matches_brute_force():
    rng = np.random.default_rng(7)
    for _ in range(20):
        n = int(rng.integers(1, 60))
        arr = np.cumsum(rng.exponential(0.01, n))
        done = arr + rng.exponential(0.03, n)
        st = bench.serving_stats(arr, done)
        depth = [sum(1 for j in range(n) if arr[j] <= arr[i] < done[j]) for i in range(n)]
        assert st["max_queue_depth"] == max(depth)
        assert np.isclose(st["mean_queue_depth"], np.mean(depth))
        lat = (done - arr) * 1e3
        assert np.isclose(st["p99_latency_ms"], np.percentile(lat, 99))
