"""bench.py's command line on the CPU: it measures one GPU only and says so."""
from __future__ import annotations

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    for n in ("2", "8"):
        out = _bench("--gpus", n)
        assert out.returncode == 2
        assert "one GPU only" in out.stderr and f"--gpus {n}" in out.stderr
        assert out.stdout == ""  # no JSON line for a run that did not happen


def test_help_lists_every_workload():
    out = _bench("--help")
    assert out.returncode == 0
    for w in ("c2", "sweep", "fill", "zipf", "c4", "serve", "tcf", "point"):
        assert w in out.stdout
