"""The serving scheduler (bc_server.cpp) on the host, behind a stand-in
device backend: concurrent submit / poll (blocking and not) / stats threads,
expiring deadlines, admission refusals and a destroy while pollers are
blocked, run under ThreadSanitizer and under AddressSanitizer + UBSan.  Every
result must equal the stand-in's count for its query.  (clang's TSan is used:
it follows the condition-variable waits on the steady clock that the
scheduler makes.)"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CLANG = "/opt/rocm/llvm/bin/clang++"
SRC = [os.path.join(ROOT, "paper_2403_07858_amd", "csrc", "bc_server.cpp"), os.path.join(HERE, "server_stress.cpp")]
INC = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2403_07858_amd", "csrc")]


@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ of the ROCm toolchain not found")
@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_server_scheduler_under_sanitizer(tmp_path, san):
    exe = str(tmp_path / "server_stress")
    subprocess.run([CLANG, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-pthread",
                    "-fsanitize=" + san, *INC, *SRC, "-o", exe], check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, "3", "400"], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "Sanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.count("bad 0") == 3, r.stdout
