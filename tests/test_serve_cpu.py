"""The serving scheduler on the host alone: tests/serve_sched_check.cpp drives
csrc/serve_core.hpp (queue, admission by footprint into a first-fit arena, worker slots,
cancellation, statistics) with a fake executor from several submitter threads, built with g++
under ThreadSanitizer and under AddressSanitizer + UBSan.  A data race, an out-of-bounds access,
overlapping arena ranges or a ticket without a final state fails it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "serve_sched_check.cpp")
INC = [os.path.join(ROOT, "paper_2009_09767_amd", "csrc"), os.path.join(ROOT, "include")]


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_scheduler_under_sanitizer(tmp_path, san):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "serve_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fno-omit-frame-pointer", f"-fsanitize={san}",
           SRC, "-o", exe]
    for i in INC:
        cmd[1:1] = ["-I", i]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    env["ASAN_OPTIONS"] = "detect_leaks=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(p.stdout)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "ThreadSanitizer" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr
    assert "runtime error" not in p.stderr, p.stderr
