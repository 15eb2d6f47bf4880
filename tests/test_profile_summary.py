"""CPU tests of the rocprofv3 summary tool that bench.py reads its traffic
figure from: counter scaling against the copy calibration, the kernel-source
hash that voids stale counters, and the VALU-per-cell table."""
import csv
import os

import pytest

from paper_2506_03905_amd import profile_summary as PS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _counter_csv(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})
    return d


def test_code_only_drops_comments_and_spacing_keeps_strings():
    a = 'int x = 1; // note\n/* block\n comment */ const char *s = "a // b";\n'
    b = 'int   x = 1;\n\nconst char *s = "a // b"; // other note\n'
    assert PS._code_only(a) == PS._code_only(b)
    assert '"a // b"' in PS._code_only(a)
    assert PS._code_only("int x = 1;") != PS._code_only("int x = 2;")


def test_traffic_scales_counters_by_the_copy(tmp_path, monkeypatch):
    """A copy of N bytes that FETCH_SIZE reports as N/2 (KiB units) and
    WRITE_SIZE as N gives scales 2 and 1; the kernel's mean per dispatch is
    scaled by them, and the JSON block reads back while the kernel sources
    are unchanged."""
    n = 1 << 20
    cf = _counter_csv(str(tmp_path / "cf"), [("copyBuffer", "FETCH_SIZE", n / 2 / 1024)])
    cw = _counter_csv(str(tmp_path / "cw"), [("copyBuffer", "WRITE_SIZE", n / 1024)])
    kf = _counter_csv(str(tmp_path / "kf"), [("k_step<19>", "FETCH_SIZE", 100.0),
                                             ("k_step<19>", "FETCH_SIZE", 300.0),
                                             ("k_wall<3>", "FETCH_SIZE", 9e9)])
    kw = _counter_csv(str(tmp_path / "kw"), [("k_step<19>", "WRITE_SIZE", 400.0)])

    class A:
        kernel, fetch, write, copy_fetch, copy_write = "k_step", kf, kw, cf, cw
        copy_bytes, copy_kernel, algorithmic_bytes, cmd = float(n), "copyBuffer", 1000.0 * 1024, "cmd"

    text = PS.traffic(A)
    out = tmp_path / "t.md"
    out.write_text(text)
    t = PS.read_traffic(str(out))
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["fetch_bytes"] == pytest.approx(200.0 * 1024 * 2.0)   # mean of 100 and 300 KiB
    assert t["write_bytes"] == pytest.approx(400.0 * 1024)
    assert t["traffic_over_algorithmic"] == pytest.approx((400.0 * 1024 + 400.0 * 1024) / (1000.0 * 1024))
    monkeypatch.setattr(PS, "source_sha256", lambda: "other kernels")
    assert PS.read_traffic(str(out)) is None


def test_valu_per_cell(tmp_path):
    k = "_ZN12_GLOBAL__N_16k_stepILi19EffLb0ELb0ELb0ELb0ELb0ELb0EEEvN4lbmd2KPEi"
    d = _counter_csv(str(tmp_path / "v"), [(k, "SQ_INSTS_VALU", 64.0e6), (k, "SQ_WAVES", 1.0e5)])
    stats = tmp_path / "s.csv"
    with open(stats, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "AverageNs"])
        w.writeheader()
        w.writerow({"Name": k, "AverageNs": 1.0e6})

    class A:
        kernel, pmc, cells, cmd = "k_step", d, 6400000, "cmd"
    A.stats = str(stats)
    text = PS.valu(A)
    row = [line for line in text.splitlines() if line.startswith("| `")][0]
    # 640 VALU instructions per wave of 64 cells; issue 64e6 * 4 / (1024 * 2.4e9) s
    assert "| 640 |" in row
    assert f"{64.0e6 * 4 / (1024 * 2.4e9) * 1e6:.1f}" in row


def test_committed_traffic_profile_matches_the_kernels():
    """The benchmark's traffic figure comes from this summary; it must have
    been taken with the kernel sources in the tree."""
    t = PS.read_traffic(os.path.join(ROOT, "profiles", "k_step_d3q19_512x256x256_f32_traffic.md"))
    assert t is not None
    assert 1.0 <= t["traffic_over_algorithmic"] < 1.05
