"""bench.py's command line on a host without a GPU: the one-GPU rule and its argument set."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_modes_and_reports_are_listed():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--mode", "--serve-mode", "--sweep-mode", "--sigma-report", "--precision-report",
                 "--next-report", "--host-report", "--serving-sweep", "--steps", "--warmup"):
        assert flag in r.stdout, flag
    assert "hybrid" in r.stdout
