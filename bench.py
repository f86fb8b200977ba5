"""Throughput of the Yee FDTD hot path on one MI355X.

A bench "step" is one complete run of the single-shower workload (256x256x2048 cells of 1 cm,
n = 1.78, 10-cell CPML, moving Greisen-like shower, 64 FP64 observers, 4000 Yee steps), from
zero fields, as one hipGraph launch.  The value is Yee cell-updates per second (all six
components of one cell, one time step), whole job.

Prints one JSON line with the roofline of the dominant kernel (the fused E/H sweep) and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for f in ("chf_kernels.hip", "chf_internal.h"):
        with open(os.path.join(ROOT, "paper_1001_5341_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, storage: str, bytes_alg_per_launch: float):
    """HBM bytes per launch of the sweep from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_fused_sweep_{workload}_{storage}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_digest") != kernel_source_digest():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(w, seconds_hint: float = 15.0):
    """The FP64 oracle on a bounded sample of the workload: a 256x256x256 sub-grid (same
    spacing, CPML and shower source, observers shifted into it) for a few dozen steps."""
    import oracle
    from paper_1001_5341_amd import workloads as W

    nz = 256
    sub = W.greisen_shower(w.seed, w.nx, w.ny, nz, 40, 8, zmax_frac=(0.4, 0.5),
                           length_range=(0.5, 1.0), r_range=(0.3, 1.0), name="cpu-sample")
    t0 = time.perf_counter()
    oracle.run(sub)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rate = sub.n_cells * sub.n_steps / dt / 1e6
    return {"value": round(rate, 3), "unit": "Mcell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle, {sub.nx}x{sub.ny}x{sub.nz} sub-grid of the workload "
                      f"(CPML-10, shower source, 8 observers), {sub.n_steps} steps, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="single-shower")
    ap.add_argument("--storage", default="fp32", choices=["fp32", "bf16", "fp16"])
    ap.add_argument("--kernel", default="auto", choices=["auto", "fused", "split"])
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--time-steps", type=int, default=0, help="override the Yee steps per run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU z-slab decomposition is design-only)"}))
        sys.exit(2)

    import torch

    from paper_1001_5341_amd import solver
    from paper_1001_5341_amd import workloads as W

    w = W.workload_by_name(args.workload)
    if args.time_steps:
        w = w.replace(n_steps=args.time_steps)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] workload {w.name}: {w.nx}x{w.ny}x{w.nz}, {w.n_steps} steps, "
          f"storage {args.storage}", file=sys.stderr, flush=True)
    plan = solver.Plan(w, storage=args.storage, kernel=args.kernel, rows=args.rows,
                       waves=args.waves, zchunk=args.zchunk, device=dev)
    info = plan.info()
    out = plan.new_waveforms()
    stream = torch.cuda.current_stream()
    for i in range(args.warmup):
        plan.run(out=out, graph=True, sync=True)
        print(f"[bench] warmup {i} done", file=sys.stderr, flush=True)

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        plan.run(out=out, graph=True, sync=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.sync()
    gpu_ms = ev0.elapsed_time(ev1)
    print(f"[bench] timed {args.steps} runs: wall {wall:.3f} s, events {gpu_ms / 1e3:.3f} s",
          file=sys.stderr, flush=True)

    cells = w.nx * w.ny * w.nz
    updates = cells * w.n_steps * args.steps
    value = updates / wall / 1e6
    # dominant kernel: the sweep, one launch per Yee step; the event time per Yee step also
    # contains the small source and observer kernels (a few microseconds), so this is a bound
    # from below on the sweep's own rate
    step_s = gpu_ms / 1e3 / (args.steps * w.n_steps)
    b_cell = info["bytes_per_cell_update"]
    alg_bytes_launch = b_cell * cells
    achieved = alg_bytes_launch / step_s / 1e9
    traffic = measured_traffic(w.name, args.storage, alg_bytes_launch)
    rec = {
        "metric": "Yee Mcell-updates/s and % HBM roofline, FP32 vs BF16-storage at stated L2 error",
        "value": round(value, 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16-storage/f32-math", "fp16": "f16-storage/f32-math"}[args.storage],
        "data": "synthetic (seeded Greisen-like shower, no datasets)",
        "config": {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "yee_steps_per_run": w.n_steps,
                   "boundary": f"{w.bc}{w.npml}", "observers": w.n_obs, "storage": args.storage,
                   "kernel": {1: "split", 2: "fused"}[info["kernel"]],
                   "tile": {"vx": info["vx"], "rows_per_wave": info["rows_per_wave"],
                            "waves_per_block": info["waves_per_block"], "z_chunk": info["z_chunk"]},
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "bytes_per_cell_update": round(b_cell, 3),
                     "kernel": "k_fused (one launch per Yee step)",
                     "launch_avg_us": round(step_s * 1e6, 2)},
    }
    if not args.no_accuracy and w.name.startswith("single-shower") and not args.time_steps:
        gold = os.path.join(ROOT, "tests", "golden", "single-shower_oracle.npz")
        if os.path.exists(gold):
            ref = np.load(gold)["waveforms"].astype(np.float64)
            got = out.cpu().numpy()
            err = np.sqrt(((got - ref) ** 2).sum(axis=(1, 2)) / (ref ** 2).sum(axis=(1, 2)))
            rec["accuracy_vs_fp64_oracle"] = {"rel_l2_max": float(err.max()),
                                              "rel_l2_median": float(np.median(err))}
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a CPU sample", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(w)
    plan.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
