"""The bench's command-line contract on the CPU: one GPU only, and the
profiling switches it documents."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_exits_with_a_message():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_help_lists_the_profiling_switches():
    r = run_bench("--help")
    assert r.returncode == 0
    for opt in ("--headline-only", "--widened-only", "--batch-only", "--write-traffic", "--budget-s"):
        assert opt in r.stdout
