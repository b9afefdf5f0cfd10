"""CPU model of the enumeration kernel's subtask ring (runtime split of heavy
tasks): every task and queued subtask runs exactly once and every worker
leaves the drain loop, with ThreadSanitizer watching the memory orders."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("split") / "split_sim")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=thread", "-pthread",
                    os.path.join(HERE, "split_protocol_sim.cpp"), "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("threads,tasks,cap", [(16, 20000, 5000), (8, 3000, 100000), (32, 5000, 64), (3, 10, 4)])
def test_every_subtask_runs_once_and_workers_exit(sim, threads, tasks, cap):
    r = subprocess.run([sim, str(threads), str(tasks), str(cap)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ThreadSanitizer" not in r.stderr, r.stderr
    assert "errors 0" in r.stdout
