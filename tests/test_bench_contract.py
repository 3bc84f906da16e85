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
                "--serve-rates", "--no-cpu-baseline", "--calibrate-copy", "--alphas",
                "--serve-queries", "--queries"):
        assert opt in p.stdout, opt


def test_traffic_only_for_the_profiled_expansion_source(tmp_path, monkeypatch):
    """`roofline.traffic` comes from a stored counter record only while the
    expansion source of the timed path is byte-identical to the one the
    counters were taken on, and only for the edge-mode run they describe."""
    import hashlib
    import json
    import types

    sys.path.insert(0, ROOT)
    import bench
    csrc = tmp_path / "paper_2001_06770_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    for kern, src_name, path in (("k_expand", "explore.hip", "single"),
                                 ("k_co_expand", "cohort.hip", "batched")):
        src = f"// {kern}\n".encode()
        (csrc / src_name).write_bytes(src)
        key = src_name.replace(".", "_") + "_sha256"
        rec = {"bytes_per_launch": 1234.0, key: hashlib.sha256(src).hexdigest()}
        (tmp_path / "profiles" / f"{kern}_medium_traffic.json").write_text(json.dumps(rec))
        monkeypatch.setattr(bench, "ROOT", str(tmp_path))
        args = types.SimpleNamespace(workload="medium", path=path, mode="edge")
        assert bench.traffic_for(args) == 1234.0
        assert bench.traffic_for(types.SimpleNamespace(workload="large", path=path,
                                                       mode="edge")) is None
        assert bench.traffic_for(types.SimpleNamespace(workload="medium", path=path,
                                                       mode="node")) is None
        (csrc / src_name).write_bytes(src + b"// changed\n")
        assert bench.traffic_for(args) is None


def test_algorithmic_bytes_model():
    """The roofline's bytes follow the stated per-run model."""
    sys.path.insert(0, ROOT)
    import bench
    st = [{"levels": 3, "e_arc": 100, "gate_pass": 40, "h_writes": 7, "frontier": 9},
          {"levels": 0, "e_arc": 0, "gate_pass": 0, "h_writes": 0, "frontier": 0}]
    e, lp = bench.alg_bytes(st, 2, 3, 80)
    assert e == 5 * 100 + 2 * 40 + 7
    assert lp == e + (4 + 8 + 2) * 9 + 3 * 80 / 8 + 80 * 2
