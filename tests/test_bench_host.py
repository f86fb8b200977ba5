"""Host logic of bench.py, without a GPU: the refusal of more than one GPU, the calibration
arithmetic of the counter summary, the traffic lookup keyed by kernel source and tile shape, the
roofline figures and the waveform error metrics."""
import json
import os
import subprocess
import sys
import types

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def _csv(path, counter, rows):
    with open(path, "w") as fh:
        fh.write("Kernel_Name,Grid_Size,Counter_Name,Counter_Value\n")
        for name, value in rows:
            fh.write(f'"{name}",4096,{counter},{value}\n')


def test_counter_summary_calibration_and_traffic_lookup(tmp_path, monkeypatch):
    """FETCH_SIZE of the 256 MiB calibration copy reads half its bytes (factor 2), WRITE_SIZE all
    of them (factor 1); the sweep's per-dispatch mean is scaled by those factors, and the record
    is found again only for the tile shape (and kernel sources) it was taken on."""
    fused = "void chf::k_fused<float, 4, 8, true>(chf::Dev, chf::FusedShape, int)"
    other = "void chf::k_fused_gen<float, 4, 8, 1, false>(chf::Dev, chf::FusedShape, int const*, int, int)"
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _csv(f, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 12.0), ("__amd_rocclr_copyBuffer", 131072.0),
                           (fused, 1000.0), (fused, 1200.0), (other, 77777.0)])
    _csv(w, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 262144.0), (fused, 500.0), (fused, 500.0)])
    monkeypatch.setattr(bench, "traffic_path", lambda wl, st: str(tmp_path / f"traffic_{wl}_{st}.json"))
    tile = [8, 12, "fused_prefetch"]
    bench.summarize_pmc(str(f), str(w), "single-shower", "fp32", "cmd", tile)
    rec = json.load(open(tmp_path / "traffic_single-shower_fp32.json"))
    assert rec["fetch"]["scale"] == 2.0 and rec["write"]["scale"] == 1.0
    assert rec["fetch"]["dispatches"] == 2
    assert rec["fetch"]["bytes_per_launch"] == 1100.0 * 1024 * 2.0
    assert rec["write"]["bytes_per_launch"] == 500.0 * 1024
    assert rec["bytes_per_launch"] == 1100.0 * 1024 * 2.0 + 500.0 * 1024
    assert rec["kernel_digest"] == bench.kernel_digest_for("single-shower")
    assert bench.measured_traffic("single-shower", "fp32", tile) == rec["bytes_per_launch"]
    assert bench.measured_traffic("single-shower", "fp32", [7, 8, "fused"]) is None
    rec["kernel_digest"] = "0" * 16  # kernels changed since the counters were taken
    json.dump(rec, open(tmp_path / "traffic_single-shower_fp32.json", "w"))
    assert bench.measured_traffic("single-shower", "fp32", tile) is None


def test_counter_summary_of_the_two_step_sweep(tmp_path, monkeypatch):
    """With the two-step tile the counted dispatches are the two-step interior kernel's, not the
    one-step sweep's."""
    step2 = "void chf::k_step2<float, 4, 8, 1>(chf::Dev, chf::Shape2, int, int, double const*)"
    fused = "void chf::k_fused<float, 4, 8, true>(chf::Dev, chf::FusedShape, int)"
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _csv(f, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 131072.0), (step2, 3000.0), (fused, 10.0)])
    _csv(w, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 262144.0), (step2, 700.0), (fused, 10.0)])
    monkeypatch.setattr(bench, "traffic_path", lambda wl, st: str(tmp_path / f"traffic_{wl}_{st}.json"))
    tile = [8, 32, "fused2"]
    bench.summarize_pmc(str(f), str(w), "single-shower", "fp32", "cmd", tile)
    rec = json.load(open(tmp_path / "traffic_single-shower_fp32.json"))
    assert "k_step2" in rec["kernel"]
    assert rec["bytes_per_launch"] == 3000.0 * 1024 * 2.0 + 700.0 * 1024
    assert bench.measured_traffic("single-shower", "fp32", tile) == rec["bytes_per_launch"]


def test_roofline_figures():
    r = bench.roofline({"fused_cells": 1_000_000, "fused_bytes_per_cell": 50.0}, fused_ms=10.0, yee_steps=100)
    # 50 MB per launch in 0.1 ms
    assert r["achieved"] == 500.0 and r["launch_avg_us"] == 100.0
    assert r["frac"] == round(500.0 / bench.HBM_PEAK_GBS, 4) and r["bound"] == "hbm"
    # two Yee steps per launch: 50 launches of 0.2 ms, each counting both steps' one-step bytes
    # (100 B per node), beside the pass's own 50 B per node
    r2 = bench.roofline({"fused_cells": 1_000_000, "fused_bytes_per_cell": 100.0, "pass_bytes_per_cell": 50.0,
                         "steps_per_launch": 2}, fused_ms=10.0, yee_steps=100)
    assert r2["launches"] == 50 and r2["launch_avg_us"] == 200.0 and r2["achieved"] == 500.0
    assert r2["temporal_blocking"]["pass_achieved_gbs"] == 250.0
    w = types.SimpleNamespace(nr=1000, nz=1001)
    z = bench.rz_roofline(w, ms=20.0, launches=100, spl=2)
    # 1000 x 1000 marched nodes x 24 B in 0.2 ms; two Yee steps per pass double the effective rate
    assert z["alg_bytes_per_launch"] == 1000 * 1000 * bench.RZ_BYTES_PER_NODE
    assert z["achieved"] == round(24e6 / 0.2e-3 / 1e9, 1)
    assert z["effective_single_step_gbs"] == round(2 * z["achieved"], 1)


def test_waveform_error_metrics():
    rng = np.random.default_rng(0)
    ref = rng.standard_normal((4, 3, 50))
    got = ref * (1.0 + 1e-3)
    e = bench.waveform_error(got, ref)
    assert abs(e["rel_l2_max"] - 1e-3) < 1e-12 and abs(e["rel_l2_median"] - 1e-3) < 1e-12
    assert abs(e["peak_amp_err_max"] - 1e-3) < 1e-12
    got2 = ref.copy()
    got2[2] *= 1.01
    e2 = bench.waveform_error(got2, ref)
    assert abs(e2["rel_l2_max"] - 1e-2) < 1e-12 and e2["rel_l2_median"] == 0.0


def test_traffic_records_are_found_under_the_short_workload_names():
    """The bench is run with short workload names ("precision", "single-shower"); the counter
    records are named for the full workload, so both names find the same committed record."""
    p = bench.traffic_path("precision", "fp32")
    assert p.endswith("traffic_fused_sweep_precision-512x512x4096_fp32.json")
    assert p == bench.traffic_path("precision-512x512x4096", "fp32")
    assert bench.traffic_path("single-shower", "fp32") == bench.traffic_path("single-shower-256x256x2048", "fp32")
    assert bench.traffic_path("rz-8192", "fp32").endswith("traffic_rz_step_rz-8192_fp32.json")
    for wl in ("precision", "single-shower", "rz-8192"):
        assert os.path.exists(bench.traffic_path(wl, "fp32")), wl
