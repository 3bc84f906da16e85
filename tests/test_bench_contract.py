"""Benchmark command-line contract, checked without a GPU: one GPU only, and
the options the measurements rely on are there."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    p = run("--gpus", "2")
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""          # no JSON line for an unsupported run


def test_options_present():
    p = run("--help")
    assert p.returncode == 0
    for opt in ("--steps", "--warmup", "--workload", "--path", "--lanes", "--only-timed",
                "--serve-rates", "--no-cpu-baseline", "--calibrate-copy"):
        assert opt in p.stdout, opt
