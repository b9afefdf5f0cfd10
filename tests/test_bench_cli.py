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
