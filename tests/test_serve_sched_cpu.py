"""The request loop's scheduling core on the CPU, under sanitizers (no GPU).

tests/serve_sched_harness.cpp drives the step-level engines and the
batch-level workers of paper_2009_01614_amd/csrc/serve_sched.cpp with stub
runners, from several producer threads and one consumer; it checks that every
request comes back exactly once with its own answer, that each table row
sweeps every chunk exactly once, and the error and run-alone paths.  Built
once with ThreadSanitizer and once with AddressSanitizer + UndefinedBehavior-
Sanitizer (host code only: g++, no HIP).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2009_01614_amd", "csrc")


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_scheduler_under_sanitizer(tmp_path, san):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    exe = tmp_path / "harness"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", f"-fsanitize={san}", "-fno-omit-frame-pointer",
           "-I", CSRC, os.path.join(CSRC, "serve_sched.cpp"), os.path.join(ROOT, "tests", "serve_sched_harness.cpp"),
           "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert r.stdout.strip().endswith("ok")
    assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
