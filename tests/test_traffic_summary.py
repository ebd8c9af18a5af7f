"""Host logic of the traffic figures: bench.py turns two rocprofv3 counter
files (FETCH_SIZE, WRITE_SIZE per dispatch) into HBM bytes per phase launch,
calibrated by a 1 GiB copy, and keys the record by launch variant.  The
counter files here are synthetic, with values chosen so the answer is known."""
import csv
import json

import bench

KIB_GIB = (1 << 30) / 1024


def _write_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            # each dispatch's value split over two rows (per-XCD instances)
            for half in (0.25, 0.75):
                w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter,
                            "Counter_Value": value * half})


def _probe(path, variant, sweeps=10):
    with open(path, "w") as f:
        f.write("some log line\n")
        f.write(json.dumps({"probe": "qbd_L4096_m64_fp64", "variant": variant, "sweeps": sweeps,
                            "phase_a_bytes": 1000.0, "phase_b_bytes": 1000.0,
                            "copy_bytes_each_way": 1 << 30, "source_hash": "abc"}) + "\n")


def _run(tmp_path, monkeypatch, variant, kernels, fetch_copy, write_copy):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir(exist_ok=True)
    _probe(tmp_path / "probe.txt", variant)
    copy = "__amd_rocclr_copyBuffer"
    _write_csv(tmp_path / "f.csv", "FETCH_SIZE",
               [(n, f) for n, f, _ in kernels] + [(copy, fetch_copy)] * 3)
    _write_csv(tmp_path / "w.csv", "WRITE_SIZE",
               [(n, w) for n, _, w in kernels] + [(copy, write_copy)] * 3)
    bench.traffic_summary(str(tmp_path / "probe.txt"), str(tmp_path / "f.csv"),
                          str(tmp_path / "w.csv"))
    with open(tmp_path / "profiles" / "traffic.json") as f:
        return json.load(f)["qbd_L4096_m64_fp64"]


def test_per_phase_variant(tmp_path, monkeypatch):
    a = "void stc::k_sweep<double, 64, 1, false, 4, true>(stc::SweepLaunch)"
    b = "void stc::k_sweep<double, 64, 1, true, 4, true>(stc::SweepLaunch)"
    other = "void stc::k_sweep<double, 64, 1, false, 8, true>(stc::SweepLaunch)"
    # the fetch counter reads half of the copy's bytes: scale 2
    rec = _run(tmp_path, monkeypatch, 3,
               [(a, 100.0, 10.0), (b, 120.0, 12.0), (a, 100.0, 10.0), (b, 120.0, 12.0),
                (other, 9999.0, 9999.0)],
               KIB_GIB / 2, KIB_GIB)["3"]
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["bytes_per_launch"] == (100 * 2 + 10) * 1024
    assert rec["phase_b_bytes_per_launch"] == (120 * 2 + 12) * 1024
    assert rec["dispatches"] == 2


def test_persistent_variant_splits_a_burst_and_keeps_other_variants(tmp_path, monkeypatch):
    a = "void stc::k_sweep<double, 64, 1, false, 4, true>(stc::SweepLaunch)"
    b = "void stc::k_sweep<double, 64, 1, true, 4, true>(stc::SweepLaunch)"
    _run(tmp_path, monkeypatch, 3, [(a, 100.0, 10.0), (b, 120.0, 12.0)], KIB_GIB, KIB_GIB)
    flow = "void stc::k_sweep_flow<double, 64, 1, 4, true>(stc::FlowLaunch)"
    # one dispatch of 10 sweeps = 20 phases
    table = _run(tmp_path, monkeypatch, 7, [(flow, 2000.0, 400.0)], KIB_GIB, KIB_GIB)
    assert set(table) == {"3", "7"}
    rec = table["7"]
    assert rec["bytes_per_launch"] == rec["phase_b_bytes_per_launch"] == (100 + 20) * 1024
    assert rec["sweeps_per_probe"] == 10 and rec["dispatches"] == 1


def test_measured_traffic_needs_the_same_sources_and_variant(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h1")
    rec = {"w": {"3": {"source_hash": "h1", "bytes_per_launch": 5},
                 "7": {"source_hash": "h0", "bytes_per_launch": 6}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("w", 3) == 5
    assert bench.measured_traffic("w", 7) is None     # taken on other sources
    assert bench.measured_traffic("w", 1) is None     # never measured
    assert bench.measured_traffic("x", 3) is None
