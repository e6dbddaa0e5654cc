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


def test_oracle_shards_cover_every_filter_once_and_balance():
    # the all-core oracle baselines spread filters over host threads,
    # heaviest first to the least-loaded thread
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench

    w = {i: (1 << (10 + i % 11)) for i in range(300)}
    shards = bench.shard(list(w), lambda i: w[i], 16)
    flat = sorted(i for s in shards for i in s)
    assert flat == list(range(300))
    loads = [sum(w[i] for i in s) for s in shards]
    assert max(loads) - min(loads) <= max(w.values())
    assert bench.shard([], lambda i: 1, 4) == [[], [], [], []]
    assert 1 <= bench.host_threads() <= 16
