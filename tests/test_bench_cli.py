"""bench.py's command line on the CPU: one GPU only."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    """--gpus N with N > 1 ends with a message and a non-zero status before
    any device work."""
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU only" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")       # no result line
