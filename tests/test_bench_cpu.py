"""bench.py's command-line contract, without a GPU: it measures one GPU only
and says so for any other count; the committed counter figures are only
used for the kernel sources they were taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120, env=e)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_world_size_above_one_is_refused():
    r = run_bench("--steps", "1", env={"WORLD_SIZE": "2"})
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_committed_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    doc = {"source_sha256": bench.source_hash(),
           "kernels": {"k_x": {"launches": 4, "read_bytes": 300.0, "write_bytes": 100.0}}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_1g_path.json").write_text(json.dumps(doc))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: doc["source_sha256"])
    assert bench.committed_traffic("k_x") == 100
    assert bench.committed_traffic("k_missing") is None
    monkeypatch.setattr(bench, "source_hash", lambda: "other sources")
    assert bench.committed_traffic("k_x") is None
