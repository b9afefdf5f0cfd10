"""Command-line contract of bench.py that holds without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          cwd=ROOT, capture_output=True, text=True, timeout=120,
                          env={**os.environ, **(env or {})})


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_multi_rank_launch_is_refused():
    r = _bench("--gpus", "1", env={"WORLD_SIZE": "4"})
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_traffic_reported_only_for_the_measured_launch():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.traffic_bytes("power_law_20m", [(4, 4)]) is None
    assert bench.traffic_bytes(bench.TRAFFIC_WORKLOAD, [(4, 6), (6, 4)]) is None
    got = bench.traffic_bytes(bench.TRAFFIC_WORKLOAD, [(4, 4)])
    assert got is None or got == bench.TRAFFIC_BYTES_Q44


def test_range_cuts_cover_every_root_once():
    # the ranged count adds up only if the ranges tile [0, n) with no gap or
    # overlap; a heavy fine range ends up in a range of its own
    sys.path.insert(0, ROOT)
    import bench
    import numpy as np
    rng = np.random.default_rng(5)
    w = np.sort(rng.pareto(1.5, 10_000))
    for n in (1, 3, 16, 24):
        c = bench.equal_weight_cuts(w * w, n)
        assert len(c) == n + 1 and c[0] == 0 and c[-1] == len(w)
        assert all(a <= b for a, b in zip(c, c[1:]))
    fine = bench.equal_weight_cuts(w * w, 96)
    times = [1.0] * 96
    times[50] = 1000.0
    for n in (1, 4, 24):
        cuts = bench.merge_cuts(fine, times, n)
        assert cuts[0] == 0 and cuts[-1] == len(w)
        assert all(a < b for a, b in zip(cuts, cuts[1:]))
        assert set(cuts) <= set(fine) and len(cuts) <= n + 1
        if n == 24:
            assert fine[50] in cuts and fine[51] in cuts   # the heavy range alone
    assert bench.equal_weight_cuts([], 4) == [0] * 5
