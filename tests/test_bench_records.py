"""The benchmark's counter records: the HBM traffic and VALU occupancy that
`bench.py` attaches to its roofline come from committed counter passes and
are used only while the step kernel is the one that was counted."""
import json

import bench


def _write(tmp_path, name, rec):
    p = tmp_path / name
    p.write_text(json.dumps(rec))
    return str(p)


def test_valu_record_scales_counted_instructions_to_the_live_kernel_time(tmp_path, monkeypatch):
    rec = {"kernel_hash": bench.kernel_hash(), "valu_insts_per_launch": 1024 * 60000.0,
           "sample_valu_insts_per_launch": 1024 * 70000.0, "simds": 1024}
    monkeypatch.setattr(bench, "VALU_FILE", _write(tmp_path, "v.json", rec))
    v = bench.read_valu(kernel_ms=0.1, per_period=10)
    # one sample launch in ten: 61000 wave64 instructions per SIMD, 4 cycles each
    assert v["issue_cycles_per_simd"] == 244000.0
    assert abs(v["frac"] - 244000.0 / (2.4e9 * 1e-4)) < 1e-12
    rec["kernel_hash"] = "0" * 16
    monkeypatch.setattr(bench, "VALU_FILE", _write(tmp_path, "w.json", rec))
    assert bench.read_valu(kernel_ms=0.1, per_period=10) is None


def test_traffic_record_is_dropped_when_the_kernel_changed(tmp_path, monkeypatch):
    rec = {"kernel_hash": bench.kernel_hash(), "hbm_bytes_per_launch": 5.5e8}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _write(tmp_path, "t.json", rec))
    assert bench.read_traffic(1) == 5.5e8
    rec["kernel_hash"] = "f" * 16
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _write(tmp_path, "u.json", rec))
    assert bench.read_traffic(1) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.read_traffic(1) is None
