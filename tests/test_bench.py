"""Host-side checks of bench.py: the one-GPU guard and the traffic record."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _record(tmp_path, sha, workload):
    rec = {"source_sha256": sha, "workload": workload,
           "forms": {"split3_bf16": {"fetch_bytes": 4.0e9, "write_bytes": 5.0e8}}}
    path = tmp_path / "rec.json"
    path.write_text(json.dumps(rec))
    return str(path)


def test_traffic_record_used_only_for_same_sources_and_workload(tmp_path, monkeypatch):
    w = {"M": 8192, "Kd": 8192, "N": 8192, "p": 64, "K": 2}
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", _record(tmp_path, bench.kernel_source_sha256(), w))
    assert bench.recorded_traffic("split3_bf16", 8192, 8192, 8192, 64, 2) == 4.5e9
    assert bench.recorded_traffic("split3_bf16", 8192, 8192, 8192, 64, 4) is None   # other schedule
    assert bench.recorded_traffic("f32", 8192, 8192, 8192, 64, 2) is None           # no record
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", _record(tmp_path, "0" * 64, w))
    assert bench.recorded_traffic("split3_bf16", 8192, 8192, 8192, 64, 2) is None   # kernels changed
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(tmp_path / "missing.json"))
    assert bench.recorded_traffic("split3_bf16", 8192, 8192, 8192, 64, 2) is None


def test_default_schedule_per_workload(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    assert bench.parse().K == 2
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", "nbody"])
    a = bench.parse()
    assert (a.K, a.p, a.bodies) == (8, 64, 1 << 18)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", "nbody", "--K", "4"])
    assert bench.parse().K == 4
    assert bench.VALU_F32_PEAK == 157.3
