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


def test_large_block_traffic(tmp_path, monkeypatch):
    """The large-block probe: apply launches per phase (the last `sweeps`
    dispatches of each), gathers apart, other kernels ignored, both counters
    calibrated by the copies; the record goes under the probe's key with its
    source hash, and the line's reader takes it only for the current
    sources."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    with open(tmp_path / "probe.txt", "w") as f:
        f.write(json.dumps({"probe": bench.LARGE_PROBE, "variant": 2, "sweeps": 2,
                            "apply_a_bytes": 1000.0 * 1024, "apply_b_bytes": 2000.0 * 1024,
                            "copy_bytes_each_way": 1 << 30, "source_hash": "abc"}) + "\n")
    aa = "void stc::k_apply_big<double, 2048, false, true>(stc::SweepLaunch, double const*)"
    ab = "void stc::k_apply_big<double, 2048, true, true>(stc::SweepLaunch, double const*)"
    ga = ("void stc::k_gather_big<double, 2048, false, true>(stc::SweepLaunch, "
          "stc::GenEntry const*, double const*, int const*, double*)")
    f32 = "void stc::k_apply_big<float, 2048, false, true>(stc::SweepLaunch, float const*)"
    copy = "__amd_rocclr_copyBuffer"
    # an autotuner trial first (dropped: only the last two dispatches count)
    fetch = [(aa, 9999.0), (aa, 500.0), (ab, 1000.0), (ga, 40.0), (aa, 500.0), (ab, 1000.0),
             (ga, 40.0), (f32, 7777.0)] + [(copy, KIB_GIB / 2)] * 3
    write = [(aa, 9999.0), (aa, 10.0), (ab, 20.0), (ga, 4.0), (aa, 10.0), (ab, 20.0),
             (ga, 4.0), (f32, 7777.0)] + [(copy, KIB_GIB)] * 3
    _write_csv(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _write_csv(tmp_path / "w.csv", "WRITE_SIZE", write)
    bench.large_traffic(str(tmp_path / "probe.txt"), str(tmp_path / "f.csv"),
                        str(tmp_path / "w.csv"))
    with open(tmp_path / "profiles" / "traffic.json") as f:
        rec = json.load(f)[f"large_{bench.LARGE_PROBE}_fp64"]
    assert rec["source_hash"] == "abc" and rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    a, b, g = (rec["launches"][k] for k in ("apply_big_a", "apply_big_b", "gather_big_a"))
    assert a["dispatches"] == 2 and a["hbm_bytes"] == (500 * 2 + 10) * 1024
    assert a["ratio"] == round((500 * 2 + 10) / 1000, 4)
    assert b["hbm_bytes"] == (1000 * 2 + 20) * 1024 and b["ratio"] == round(2020 / 2000, 4)
    assert g["hbm_bytes"] == (40 * 2 + 4) * 1024 and "ratio" not in g
    assert bench.large_traffic_record() is None          # not the current sources
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    assert bench.large_traffic_record()["apply_big_a"]["hbm_bytes"] == (500 * 2 + 10) * 1024
