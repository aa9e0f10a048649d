"""bench.py refuses, before touching a device, the runs it does not measure:
more than one GPU, and C2PLU pivoting on the batched and serving workloads."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("args", [["--gpus", "2"],
                                  ["--workload", "batched4096", "--pivoting", "c2plu"],
                                  ["--workload", "serve", "--pivoting", "c2plu"]])
def test_bench_refuses(args):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2, (r.returncode, r.stderr[-500:])
    assert r.stdout.strip() == ""
