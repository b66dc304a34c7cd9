"""Host-side logic of bench.py, without a GPU: the one-GPU contract, and the records that turn
rocprofv3 counter runs into HBM bytes and VALU instruction counts per launch (the scaling by a
plain copy of known size, and the kernel-source hash that retires a record once the kernel
changes)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
DOM = "void vpm::(anonymous namespace)::k_fixed_cells<576, unsigned short, true, 1>(vpm::FixedArgs)"
COPY = "__amd_rocclr_copyBuffer"


def _csv(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (k, c, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_traffic_record_scales_by_the_copy(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    # two launches of the dominant kernel (other kernels ignored), and a copy of COPY_BYTES
    _csv(tmp_path / "f", [(DOM, "FETCH_SIZE", 1000.0), (DOM, "FETCH_SIZE", 3000.0), ("other", "FETCH_SIZE", 9e9)])
    _csv(tmp_path / "w", [(DOM, "WRITE_SIZE", 500.0), (DOM, "WRITE_SIZE", 500.0)])
    _csv(tmp_path / "cf", [(COPY, "FETCH_SIZE", bench.COPY_BYTES / 2048.0), ("__amd_rocclr_fillBufferAligned", "FETCH_SIZE", 7.0)])
    _csv(tmp_path / "cw", [(COPY, "WRITE_SIZE", bench.COPY_BYTES / 1024.0)])
    bench.traffic_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"))
    rec = json.load(open(tmp_path / "traffic.json"))
    assert rec["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 2048.0)
    assert rec["write_bytes_per_launch"] == pytest.approx(500.0 * 1024.0)
    assert rec["launches"] == [2, 2]
    assert bench.traffic_from_profiles() == pytest.approx(2000.0 * 2048.0 + 500.0 * 1024.0)
    # a record taken on another kernel source is not used
    rec["kernel_source_sha256"] = "0" * 64
    json.dump(rec, open(tmp_path / "traffic.json", "w"))
    assert bench.traffic_from_profiles() is None


def test_valu_record(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "VALU_FILE", str(tmp_path / "valu.json"))
    rows = []
    for c, v in (("SQ_INSTS_VALU", 900.0), ("SQ_INSTS_SALU", 100.0), ("SQ_INSTS_LDS", 50.0), ("SQ_WAVES", 8.0)):
        rows += [(DOM, c, v), (DOM, c, v + 2.0), ("k_scatter<float>", c, 1e6)]
    _csv(tmp_path / "p", rows)
    bench.valu_summary(str(tmp_path / "p"))
    assert bench.valu_from_profiles() == pytest.approx(901.0)
    rec = json.load(open(tmp_path / "valu.json"))
    assert rec["sq_waves_per_launch"] == pytest.approx(9.0) and rec["launches"] == 2
    rec["kernel_source_sha256"] = "0" * 64
    json.dump(rec, open(tmp_path / "valu.json", "w"))
    assert bench.valu_from_profiles() is None

