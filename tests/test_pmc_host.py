"""Host checks of the counter reduction that turns rocprofv3 FETCH_SIZE /
WRITE_SIZE readings into HBM bytes per launch (synthetic counter files)."""
import csv
import json
import os

from paper_2406_19920_amd import pmc

COLS = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=COLS)
        w.writeheader()
        for i, (name, counter, value) in enumerate(rows):
            w.writerow({"Correlation_Id": i + 1, "Dispatch_Id": i + 1, "Kernel_Name": name,
                        "Counter_Name": counter, "Counter_Value": value})


def test_traffic_reduction(tmp_path, monkeypatch):
    zs = "void ibs::split_zgemm_kernel<16, 2>(ibs::SplitSet, int, int, int)"
    up = "void ibs::split_xgemm_kernel<16, 2, float, 2>(ibs::SplitSet, int)"
    cp = "void at::native::direct_copy_kernel(int)"
    n = 1 << 30
    # the copy reads 1.25x and writes 1.0x its bytes as counted
    _write(tmp_path / "cf", [(cp, "FETCH_SIZE", 1.25 * n / 1024)] * 3)
    _write(tmp_path / "cw", [(cp, "WRITE_SIZE", 1.0 * n / 1024)] * 3)
    _write(tmp_path / "f", [(zs, "FETCH_SIZE", 125.0), (zs, "FETCH_SIZE", 375.0), (up, "FETCH_SIZE", 50.0)])
    _write(tmp_path / "w", [(zs, "WRITE_SIZE", 100.0), (zs, "WRITE_SIZE", 300.0), (up, "WRITE_SIZE", 10.0)])
    out = tmp_path / "t.json"
    pmc.main(["--fetch", str(tmp_path / "f"), "--write", str(tmp_path / "w"),
              "--copy-fetch", str(tmp_path / "cf"), "--copy-write", str(tmp_path / "cw"),
              "--copy-bytes", str(n), "--out", str(out)])
    d = json.load(open(out))
    assert abs(d["copy_ratio"]["fetch"] - 1.25) < 1e-12 and abs(d["copy_ratio"]["write"] - 1.0) < 1e-12
    z = d["kernels"]["zgemm_split"]
    assert abs(z["fetch_bytes_per_launch"] - 250.0 * 1024 / 1.25) < 1e-6
    assert abs(z["write_bytes_per_launch"] - 200.0 * 1024) < 1e-6
    assert z["dispatches"] == [2, 2]
    assert "update" in d["kernels"] and "xgemm_split" not in d["kernels"]
    assert d["kernels"]["update"]["dispatches"] == [1, 1]
    assert pmc.traffic_for("zgemm_split", str(out)) == z["bytes_per_launch"]
    # a changed kernel source invalidates the stored figure
    d["kernels"]["zgemm_split"]["source_hash"] = "0" * 16
    json.dump(d, open(out, "w"))
    assert pmc.traffic_for("zgemm_split", str(out)) is None
    assert pmc.traffic_for("zgemm_split", str(tmp_path / "missing.json")) is None


def test_class_patterns():
    """Kernel names as rocprofv3 prints them map onto one class each."""
    import re
    names = {
        "ibs::split_xfold_kernel<8, 1, double, 0, false, 1>": "xgemm_split",
        "ibs::split_xfold_kernel<8, 1, float, 0, false, 2>": "xgemm_split",
        "ibs::split_xgemm_kernel<16, 2, double, 0>": "xgemm_split",
        "ibs::split_xfold_kernel<8, 1, float, 1, true, 1>": "update",
        "ibs::split_xfold_kernel<8, 1, float, 2, true, 2>": "update",
        "ibs::split_xfold_kernel<8, 1, float, 3, true, 1>": "update",
        "ibs::split_xfold_kernel<16, 1, float, 4, true, 2>": "update",
        "ibs::split_xgemm_kernel<16, 2, float, 4>": "update",
        "ibs::split_xgemm_kernel<16, 2, float, 2>": "update",
        "ibs::split_zfold_kernel<8, 1, true, 1>": "zgemm_split",
        "ibs::split_zgemm_kernel<16, 2>": "zgemm_split",
        "ibs::xfold_f64_kernel<1, 4, true, false>": "xgemm_f64",
        "ibs::zfold_f64_kernel<4, 1, false, true>": "zgemm_f64",
        "ibs::tridiag_kernel<float, float, 8, 9>": "tridiag_f32",
        "ibs::tridiag_kernel<double, double, 8, 9>": "tridiag_f64",
        "ibs::residual_f32_kernel(ibs::SplitSet, int)": "residual",
    }
    for name, cls in names.items():
        hits = [c for c, (pat, _) in pmc.CLASSES.items() if re.search(pat, "void " + name)]
        assert hits == [cls], (name, hits)
