"""Host-side checks of bench.py: the one-GPU guard and the traffic record."""
import json
import os
import subprocess
import sys

import pytest

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


def _bench_line(*args):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + list(args),
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    return json.loads(lines[0])


def _common(d, steps, warmup, unit):
    assert isinstance(d["metric"], str) and d["metric"]
    assert d["value"] > 0 and d["unit"] == unit
    assert d["n_gpus"] == 1 and d["steps"] == steps and d["warmup"] == warmup
    assert d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["scaling"] == "weak" and d["vs_baseline"] is None and d["data"] == "synthetic"
    assert isinstance(d["config"]["workload"], str) and d["config"]["workload"]
    r = d["roofline"]
    assert r["bound"] in ("mfma", "hbm", "alu") and r["peak"] > 0 and r["achieved"] > 0
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-9 and 0 < r["frac"] < 1
    assert "traffic" in r
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["value"] > 0 and c["cores"] >= 1 and c["sample"]


@pytest.mark.gpu
def test_bench_line_contract_step():
    """The default step's JSON line at a small size: every contract field,
    the roofline fraction consistent, every form's timed result checked."""
    if not _gpu():
        pytest.skip("no GPU")
    d = _bench_line("--n", "1024", "--p", "8", "--steps", "2", "--warmup", "1", "--cpu-seconds", "0.5")
    _common(d, 2, 1, "TFLOP/s")
    assert d["dtype"] == "split3_bf16" and d["config"]["form"] == "split3_bf16"
    assert set(d["comparison"]) == {"f32", "split2_f16"}
    for form in ("split3_bf16", "f32", "split2_f16"):
        a = d["accuracy"][form]
        for out in ("C", "dA", "dB"):
            assert a[out]["err_row"] <= 1e-5 and a[out]["err_term_u"] <= 16, (form, out, a[out])


@pytest.mark.gpu
@pytest.mark.parametrize("args,unit,steps", [
    (("--workload", "gemv", "--n", "2048", "--K", "8"), "GB/s", 200),
    (("--workload", "nbody", "--bodies", "4096"), "Ginteractions/s", 10),
    (("--workload", "complex", "--n", "512", "--p", "8"), "TFLOP/s", 10),
])
def test_bench_line_contract_workloads(args, unit, steps):
    if not _gpu():
        pytest.skip("no GPU")
    d = _bench_line(*(args + ("--cpu-seconds", "0.5")))
    _common(d, steps, 3, unit)
    assert d["accuracy"]


def _gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
