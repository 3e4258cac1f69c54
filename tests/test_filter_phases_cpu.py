"""The filter pass's phase enumeration on the CPU (no GPU).

tests/filter_phases_harness.cpp includes csrc/query_kernels.h and checks, for
every tile count up to three sample groups and random larger ones, that the
first phase (sample units) with the rest, and the first phase with the second
sample and the rest, each meet every tile exactly once, and that the serving
chunks' phase-3 tiles partition the tiles outside the sample units: every
series is compared with every query exactly once whichever phases run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2009_01614_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_filter_phases_partition_the_tiles(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("no hipcc")
    exe = tmp_path / "phases"
    cmd = [HIPCC, "-std=c++17", "-O1", "-x", "hip", "--offload-arch=gfx950", "-I", CSRC,
           os.path.join(ROOT, "tests", "filter_phases_harness.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert r.stdout.strip().endswith("ok")
