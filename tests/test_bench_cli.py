"""bench.py's contract pieces that need no GPU."""
import json
import os
import subprocess
import sys

from conftest import ROOT


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_fused_bytes_per_point():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.fused_bytes(3, 8) == 816
    assert bench.fused_bytes(3, 4) == 408
    assert bench.fused_bytes(1, 8) == 144
    assert bench.fused_bytes(2, 8) == 392


def test_traffic_record_is_tied_to_the_kernel_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    from paper_1809_09851_amd import traffic
    rec = {"kernel_hash": traffic.kernel_hash(), "n": 1 << 24, "bytes_per_launch": 1.0}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(p))
    assert bench.measured_traffic(1 << 24) == 1.0
    assert bench.measured_traffic(1 << 20) is None
    rec["kernel_hash"] = "stale"
    p.write_text(json.dumps(rec))
    assert bench.measured_traffic(1 << 24) is None


def test_traffic_record_from_counter_files(tmp_path):
    """Counters scaled by the copy probe's: a kernel that reads 40 and writes
    776 bytes per point over 2^20 points gives back exactly those bytes."""
    from paper_1809_09851_amd import traffic
    n = 1 << 20
    rows = {"fetch": [("k_fused<3>", 40 * n / 1024 / 2), ("k_copy", (1 << 30) / 1024 / 2)] * 3,
            "write": [("k_fused<3>", 776 * n / 1024), ("k_copy", (1 << 30) / 1024)] * 3}
    paths = {}
    for kind, rs in rows.items():
        p = tmp_path / f"{kind}.csv"
        p.write_text("Kernel_Name,Counter_Value\n" + "".join(f"{k},{v}\n" for k, v in rs))
        paths[kind] = str(p)
    rec = traffic.build_record("k_fused", paths["fetch"], paths["write"], n)
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    assert abs(rec["bytes_per_launch"] - 816 * n) < 1e-6 * 816 * n


def test_box_state_reads_the_driver_files(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    dev = tmp_path / "card0" / "device"
    (dev / "hwmon" / "hwmon3").mkdir(parents=True)
    (dev / "vendor").write_text("0x1002\n")
    (dev / "current_memory_partition").write_text("NPS1\n")
    (dev / "current_compute_partition").write_text("SPX\n")
    (dev / "pp_dpm_mclk").write_text("0: 900Mhz \n1: 2000Mhz *\n")
    (dev / "pp_dpm_sclk").write_text("0: 500Mhz \n1: 158Mhz *\n2: 2400Mhz \n")
    (dev / "hwmon" / "hwmon3" / "power1_cap").write_text("1400000000\n")
    (dev / "mem_info_vram_total").write_text(str(288 * 2 ** 30) + "\n")
    (dev / "mem_info_vram_used").write_text(str(3 * 2 ** 29) + "\n")
    (dev / "ras").mkdir()
    (dev / "ras" / "gpu_vram_bad_pages").write_text("0x1 : 0x1000 : R\n0x2 : 0x1000 : R\n")
    (dev / "pp_dpm_fclk").write_text("0: 1200Mhz *\n1: 2000Mhz \n")
    other = tmp_path / "card1" / "device"
    other.mkdir(parents=True)
    (other / "vendor").write_text("0x8086\n")
    s = bench.box_state(str(tmp_path))
    assert s["memory_partition"] == "NPS1" and s["compute_partition"] == "SPX"
    assert s["hbm_clock"] == "2000Mhz"
    assert s["gfx_clock_levels"] == ["500Mhz", "158Mhz", "2400Mhz"]
    assert s["power_cap_w"] == 1400.0 and s["vram_gib"] == 288.0
    assert s["vram_used_at_start_gib"] == 1.5 and s["retired_vram_pages"] == 2
    assert s["fabric_clock"] == "1200Mhz"
    assert bench.box_state(str(tmp_path / "none")) is None
