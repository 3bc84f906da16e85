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


def test_traffic_only_for_the_profiled_expansion_source(tmp_path, monkeypatch):
    """`roofline.traffic` comes from a stored counter record only while the
    expansion source is byte-identical to the one the counters were taken on,
    and only for the single-query, edge-mode run they describe."""
    import hashlib
    import json
    import types

    sys.path.insert(0, ROOT)
    import bench

    csrc = tmp_path / "paper_2001_06770_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = b"// expansion kernels\n"
    (csrc / "explore.hip").write_bytes(src)
    rec = {"bytes_per_launch": 1234.0, "explore_hip_sha256": hashlib.sha256(src).hexdigest()}
    (tmp_path / "profiles" / "k_expand_medium_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    args = types.SimpleNamespace(workload="medium", path="single", mode="edge")
    assert bench.traffic_for(args) == 1234.0
    assert bench.traffic_for(types.SimpleNamespace(workload="large", path="single", mode="edge")) is None
    assert bench.traffic_for(types.SimpleNamespace(workload="medium", path="batched", mode="edge")) is None
    assert bench.traffic_for(types.SimpleNamespace(workload="medium", path="single", mode="node")) is None
    (csrc / "explore.hip").write_bytes(src + b"// changed\n")
    assert bench.traffic_for(args) is None
