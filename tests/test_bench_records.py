"""The benchmark's counter records: the VALU instruction counts and HBM bus
bytes that `bench.py` attaches to its roofline come from committed counter
passes and are used only while the step kernel is the one that was counted
(its hash), and the closed forms the error leg checks against."""
import json

import numpy as np

import bench
import theory

VARIANT = "she_k2d_f32x8.hip"


def _write(tmp_path, name, rec):
    (tmp_path / name).write_text(json.dumps(rec))


def test_valu_record_gives_the_alu_roofline(tmp_path, monkeypatch):
    rec = {"kernel_hash": bench.kernel_hash(VARIANT), "valu_insts_per_launch": 1024 * 60000.0,
           "sample_valu_insts_per_launch": 1024 * 70000.0, "simds": 1024}
    _write(tmp_path, "v.json", rec)
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    r = bench.roofline(0.05, 1000, 2, 10, "k", VARIANT, "v.json", None)
    # two steps per launch: 0.1 ms, timed on launches outside sample steps:
    # 60000 wave64 instructions per SIMD, 64 lanes each, over 0.1 ms against
    # 256 x 4 x 16 lanes x 2.4 GHz; the sample launch's count beside it
    lane = 1024 * 60000.0 * 64
    assert r["bound"] == "alu" and r["unit"] == "Tlane-instr/s"
    assert abs(r["achieved"] - lane / 1e-4 / 1e12) < 1e-9
    assert r["sample_lane_instr_per_launch"] == 1024 * 70000.0 * 64
    assert abs(r["peak"] - 39.3216) < 1e-9
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
    assert r["lane_instr_per_cell_update"] == lane / 2000
    assert abs(r["hbm"]["achieved"] - 8.0 * 2000 / 1e-4 / 1e9) < 1e-9
    rec["kernel_hash"] = "0" * 16
    _write(tmp_path, "v.json", rec)
    r = bench.roofline(0.05, 1000, 2, 10, "k", VARIANT, "v.json", None)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["frac"] == r["hbm"]["frac"]


def test_traffic_record_is_dropped_when_the_kernel_changed(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    _write(tmp_path, "t.json", {"kernel_hash": bench.kernel_hash(VARIANT), "hbm_bytes_per_launch": 5.5e8})
    r = bench.roofline(0.05, 1000, 2, 10, "k", VARIANT, None, "t.json")
    assert r["traffic"] == 5.5e8 and abs(r["hbm"]["bus_achieved"] - 5.5e8 / 1e-4 / 1e9) < 1e-6
    _write(tmp_path, "t.json", {"kernel_hash": "f" * 16, "hbm_bytes_per_launch": 5.5e8})
    assert bench.roofline(0.05, 1000, 2, 10, "k", VARIANT, None, "t.json")["traffic"] is None
    assert bench.roofline(0.05, 1000, 2, 10, "k", VARIANT, None, "missing.json")["traffic"] is None
    assert bench.kernel_hash(VARIANT) != bench.kernel_hash("she_k3d_f32.hip")


def test_closed_forms_of_the_error_leg():
    for r, ns in ((0.1, (64, 32)), (0.05, (8, 8, 8)), (0.2, (64,))):
        g, b, h = bench.gamma_beta(r, ns)
        gt, bt = theory.gamma_beta(r, ns)
        assert abs(g - gt) < 1e-13 and abs(b - bt) < 1e-13
        want, cnt = theory.radial_average(theory.h_fe(theory.mode_x(r, ns)), ns)
        got, c2 = bench.shell_mean(h, ns)
        ok = cnt > 0
        ok[0] = False
        np.testing.assert_allclose(got[ok], want[ok] / cnt[ok], rtol=1e-13)
        np.testing.assert_array_equal(c2, cnt)


def test_copy_reference_fractions():
    roof = {"hbm": {"achieved": 6000.0, "bus_achieved": 3000.0}}
    bench.add_copy_reference(roof, 5000.0)
    h = roof["hbm"]
    assert h["copy_achieved"] == 5000.0
    assert abs(h["frac_of_copy"] - 1.2) < 1e-15 and abs(h["bus_frac_of_copy"] - 0.6) < 1e-15
    roof = {"hbm": {"achieved": 1000.0}}
    bench.add_copy_reference(roof, 4000.0)
    assert roof["hbm"]["frac_of_copy"] == 0.25 and "bus_frac_of_copy" not in roof["hbm"]
