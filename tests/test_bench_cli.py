"""bench.py's contract pieces that need no GPU: the one-GPU exit, the CPU baseline record and
the HBM traffic summary (parsed from rocprofv3 counter CSVs)."""

import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single MI355X" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


@pytest.mark.parametrize("workload", ["er60-mvc", "planted-pvc"])
def test_cpu_baseline_record(oracle_lib, monkeypatch, workload):
    monkeypatch.setattr(bench, "CPU_SAMPLE_S", 0.2)
    insts, _ = bench.instances(workload)
    r = bench.cpu_baseline(workload, insts)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["unit"] == "nodes/s"
    assert r["value"] > 0 and r["instances_per_s"] > 0 and r["seconds"] >= 0.2
    assert "passes" in r["sample"]
    json.dumps(r)


def _counter_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_traffic_summary_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    """FETCH_SIZE / WRITE_SIZE of the traversal dispatches, each scaled by what the counter reads
    for the calibration kernel that moves COPY_BYTES each way."""
    fetch = tmp_path / "fetch" / "x" / "1_counter_collection.csv"
    write = tmp_path / "write" / "x" / "1_counter_collection.csv"
    unit_f, unit_w = 2048.0, 1024.0  # bytes per counter unit
    _counter_csv(str(fetch), [
        {"Kernel_Name": "vectorized_elementwise_kernel", "Counter_Name": "FETCH_SIZE",
         "Counter_Value": bench.COPY_BYTES / unit_f},
        {"Kernel_Name": "void vc::traverse_kernel<true, false, false, false>(vc::Params)",
         "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000.0},
        {"Kernel_Name": "void vc::traverse_kernel<true, false, false, false>(vc::Params)",
         "Counter_Name": "FETCH_SIZE", "Counter_Value": 3000.0}])
    _counter_csv(str(write), [
        {"Kernel_Name": "vectorized_elementwise_kernel", "Counter_Name": "WRITE_SIZE",
         "Counter_Value": bench.COPY_BYTES / unit_w},
        {"Kernel_Name": "void vc::traverse_kernel<true, false, false, false>(vc::Params)",
         "Counter_Name": "WRITE_SIZE", "Counter_Value": 50.0},
        {"Kernel_Name": "void vc::traverse_kernel<true, false, false, false>(vc::Params)",
         "Counter_Name": "WRITE_SIZE", "Counter_Value": 150.0}])
    out = tmp_path / "summary.md"
    monkeypatch.setattr(bench, "traffic_path", lambda w: str(out))
    bench.summarize_traffic("planted-pvc", str(tmp_path / "fetch"), str(tmp_path / "write"))
    doc = json.loads(out.read_text().split("```json", 1)[1].split("```", 1)[0])
    assert doc["FETCH_SIZE"]["bytes_per_launch"] == pytest.approx(2000.0 * unit_f)
    assert doc["WRITE_SIZE"]["bytes_per_launch"] == pytest.approx(100.0 * unit_w)
    assert doc["hbm_bytes_per_launch"] == pytest.approx(2000.0 * unit_f + 100.0 * unit_w)
    assert doc["kernel_source_hash"] == bench.kernel_source_hash()
    assert bench.measured_traffic("planted-pvc") == pytest.approx(doc["hbm_bytes_per_launch"])
