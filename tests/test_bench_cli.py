"""Host-side checks of the benchmark script (no device work): the one-GPU
contract and the rule that stored HBM traffic is reported only for the kernel
sources it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    kname = "k_spmv_v<double, 2, 4, 10, true, 0>"
    rec = {"voronoi16384_k3_v": {kname: {"bytes_per_launch": 123, "source_digest": bench.kernel_source_digest()}}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("voronoi16384_k3_v", kname) == 123
    assert bench.measured_traffic("hex32_k3_vp", kname) is None
    rec["voronoi16384_k3_v"][kname]["source_digest"] = "0" * 16
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic("voronoi16384_k3_v", kname) is None
