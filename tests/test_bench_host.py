"""Host logic of bench.py's traffic figures (CPU only): the scaling of
rocprofv3 FETCH_SIZE / WRITE_SIZE counters by a copy of known size, the
per-class grouping of kernel instantiations, and the source-hash gate that
drops a traffic figure once its kernel's source has changed."""
import csv
import json
import os

import bench


def _counters(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Value": value})


def _profile_dir(tmp_path):
    d = tmp_path / "prof"
    copy = "__amd_rocclr_copyBuffer"
    # the 1 GiB copy reads twice its size and writes its size once
    _counters(str(d / "cfetch" / "c_counter_collection.csv"), [(copy, 2 * 1048576.0)])
    _counters(str(d / "cwrite" / "c_counter_collection.csv"), [(copy, 1048576.0)])
    lds = "void acr::(anonymous namespace)::k_jacobi<float, true, 1024>(acr::SvdTask const*, double, int*)"
    small = "void acr::(anonymous namespace)::k_jacobi<float, true, 256>(acr::SvdTask const*, double, int*)"
    _counters(str(d / "fetch" / "f_counter_collection.csv"), [(lds, 100.0), (lds, 300.0), (small, 200.0)])
    _counters(str(d / "write" / "w_counter_collection.csv"), [(lds, 40.0), (lds, 60.0), (small, 50.0)])
    return d


def test_summarize_pmc_scales_by_the_copy_and_groups_instantiations(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    bench.summarize_pmc(str(_profile_dir(tmp_path)), "synthetic counters")
    rec = json.loads(out.read_text())
    cal = rec["calibration"]
    assert abs(cal["scale_fetch"] - 0.5) < 1e-12 and abs(cal["scale_write"] - 1.0) < 1e-12
    cls = rec["classes"]["jacobi_lds"]
    # both instantiations in one class: 3 dispatches, mean 200 KiB read, 50 KiB written
    assert cls["dispatches"] == 3
    assert cls["fetch_kib_per_dispatch"] == 200.0 and cls["write_kib_per_dispatch"] == 50.0
    assert abs(cls["bytes_per_launch"] - (200.0 * 0.5 + 50.0 * 1.0) * 1024) < 1e-6
    # classes without dispatches in the run are left out
    assert "gemm" not in rec["classes"]


def test_traffic_is_dropped_when_the_kernel_source_changes(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    bench.summarize_pmc(str(_profile_dir(tmp_path)), "synthetic counters")
    assert abs(bench.measured_traffic("jacobi_lds") - 150.0 * 1024) < 1e-6
    rec = json.loads(out.read_text())
    rec["classes"]["jacobi_lds"]["sha256"] = "0" * 64
    out.write_text(json.dumps(rec))
    assert bench.measured_traffic("jacobi_lds") is None
    assert bench.measured_traffic("no_such_class") is None
