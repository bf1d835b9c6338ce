"""bench.py's contract pieces that need no GPU: the one-GPU exit, the CPU baseline records,
the counter summary (parsed from rocprofv3 counter CSVs) and the roofline built from it."""

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


def test_cpu_baseline_hard_families(oracle_lib, monkeypatch):
    """hard-mvc's baseline: one whole search per family, nodes/s per family and over both."""
    import graphs as G
    monkeypatch.setattr(bench, "hard_sample", lambda: [
        ("5-regular n=20", 1, G.random_regular(20, 5, 1)), ("G(24, 0.2)", 2, G.erdos_renyi(24, 0.2, 2))])
    r = bench.cpu_baseline("hard-mvc", [])
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["unit"] == "nodes/s"
    assert set(r["families"]) == {"5-regular n=20", "G(24, 0.2)"}
    total = sum(f["nodes"] for f in r["families"].values())
    assert r["value"] == pytest.approx(total / r["seconds"], rel=0.05)
    for f in r["families"].values():
        assert f["nodes"] > 0 and f["nodes_per_s"] > 0
    json.dumps(r)


def _counter_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


TRAV2 = "void vc::bitset_traverse_kernel<2, false, false, false>(vc::Params)"
TRAV3 = "void vc::bitset_traverse_kernel<3, false, false, false>(vc::Params)"


def _dispatches(counter, values, copy_value):
    """A trial launch of each kernel (to be ignored), then the call's two launches, then the
    calibration kernel, as rocprofv3 lists them."""
    rows = []
    kernels = [TRAV2, TRAV3, TRAV2, TRAV3]
    for i, (k, v) in enumerate(zip(kernels, [999.0, 999.0] + list(values))):
        rows.append({"Dispatch_Id": i + 1, "Kernel_Name": k, "Counter_Name": counter,
                     "Counter_Value": v})
    rows.append({"Dispatch_Id": 10, "Kernel_Name": "vectorized_elementwise_kernel",
                 "Counter_Name": counter, "Counter_Value": copy_value})
    return rows


def test_profile_summary_takes_the_last_call(tmp_path, monkeypatch):
    """FETCH_SIZE / WRITE_SIZE of the last call's traversal launches, each scaled by what the
    counter reads for the calibration kernel (COPY_BYTES each way); SQ counters of the same
    launches per node; trial launches before them are ignored."""
    unit_f, unit_w = 2048.0, 1024.0  # bytes per counter unit
    _counter_csv(str(tmp_path / "f" / "x" / "1_counter_collection.csv"),
                 _dispatches("FETCH_SIZE", [1000.0, 3000.0], bench.COPY_BYTES / unit_f))
    _counter_csv(str(tmp_path / "w" / "x" / "1_counter_collection.csv"),
                 _dispatches("WRITE_SIZE", [50.0, 150.0], bench.COPY_BYTES / unit_w))
    sq1, sq2 = [], []
    for name in bench.SQ_SETS[0]:
        v = 8 * 1000.0 if name == "GRBM_GUI_ACTIVE" else 600.0
        sq1 += _dispatches(name, [v, v], 1.0)
    for name in bench.SQ_SETS[1]:
        v = 8 * 1000.0 if name == "GRBM_GUI_ACTIVE" else 300.0
        sq2 += _dispatches(name, [v, v], 1.0)
    _counter_csv(str(tmp_path / "s1" / "x" / "1_counter_collection.csv"), sq1)
    _counter_csv(str(tmp_path / "s2" / "x" / "1_counter_collection.csv"), sq2)
    probe = tmp_path / "probe.json"
    probe.write_text(json.dumps({"nodes": 100, "kernel_ms": 1.0, "launches_per_call": 2,
                                 "config": {}}))
    out = tmp_path / "summary.md"
    monkeypatch.setattr(bench, "profile_path", lambda w: str(out))
    bench.summarize_profile("hard-mvc", str(probe), str(tmp_path / "f"), str(tmp_path / "w"),
                            [str(tmp_path / "s1"), str(tmp_path / "s2")])
    doc = json.loads(out.read_text().split("```json", 1)[1].split("```", 1)[0])
    assert doc["FETCH_SIZE"]["bytes_per_call"] == pytest.approx(4000.0 * unit_f)
    assert doc["WRITE_SIZE"]["bytes_per_call"] == pytest.approx(200.0 * unit_w)
    assert doc["hbm_bytes_per_call"] == pytest.approx(4000.0 * unit_f + 200.0 * unit_w)
    assert doc["instructions_per_node"]["SQ_INSTS_VALU"] == pytest.approx(1200.0 / 100)
    # two launches of 1000 cycles per XCD each: 2000 cycles; 4 * 600 quad-cycles of VALU
    assert doc["cycles_per_call"] == pytest.approx(2000.0)
    assert doc["valu_busy"] == pytest.approx(4 * 600.0 / (bench.SIMDS * 2000.0))
    assert doc["kernel_source_hash"] == bench.kernel_source_hash()
    assert bench.measured_profile("hard-mvc")["hbm_bytes_per_call"] == pytest.approx(
        doc["hbm_bytes_per_call"])


def test_alu_roofline_from_the_counter_summary(monkeypatch):
    """The bitset roofline: VALU instructions per node (counters) x nodes per call / time per
    call (measured), against 614.4 G wave-instructions/s."""
    prof = {"hbm_bytes_per_call": 5.0e6, "valu_busy": 0.5, "salu_busy": 0.2, "lds_busy": 0.01,
            "instructions_per_node": {"SQ_INSTS_VALU": 400.0}}
    monkeypatch.setattr(bench, "measured_profile", lambda w: prof)
    st = {"bitset_words": 3, "launches": 2, "lds_node_bytes": 10}
    r = bench.roofline("hard-mvc", [(None, st, 0.1, 16)], 0.1, 1.0e8, 1.0e7)
    assert r["bound"] == "alu" and r["peak"] == pytest.approx(614.4)
    assert r["achieved"] == pytest.approx(400.0 * 1.0e8 / 0.1 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 614.4)
    assert r["traffic"] == 5.0e6 and r["hbm"]["algorithmic_bytes_per_call"] == 1.0e7
    monkeypatch.setattr(bench, "measured_profile", lambda w: None)
    r = bench.roofline("hard-mvc", [(None, st, 0.1, 16)], 0.1, 1.0e8, 1.0e7)
    assert r["bound"] == "hbm" and r["traffic"] is None
