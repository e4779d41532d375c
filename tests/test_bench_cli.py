"""The benchmark's command line on a machine without a GPU: more than one GPU is refused
with a message (the multi-GPU layout is a design only), and the workloads are listed."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""          # no JSON line


def test_help_lists_the_workloads():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("c1", "c2", "c3", "c4", "c5", "c6"):
        assert w in r.stdout
