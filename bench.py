"""Throughput of the Yee FDTD hot path on one MI355X.

Default workload: the precision configuration, 512x512x4096 cells of 1 cm (n = 1.78, 10-cell
CPML, the moving Greisen-like shower, 64 FP64 observers), 6000 Yee steps per run, FP32 field
storage, with the same run in BF16 and FP16 storage beside it.  A bench "step" is one slice of
a full run: 240 consecutive Yee steps (6000 / 25), each Yee step running the H/E sweeps (fused
interior kernel plus boundary-tile kernels), the source injection and the observer gather.  The
default 25 timed steps are therefore exactly one complete run from zero fields (the fields are
zeroed before the timed region; a run that continues past 25 slices starts over from zero).
The value is Yee cell-updates per second (all six components of one cell over one time step),
whole job, inputs resident in HBM.

The timed slices go through chf_forward_timed: the same launches as chf_forward, with a hipEvent
pair on the launch stream around every launch of the dominant kernel (the fused interior
sweep), so the roofline line is that kernel's own average duration over the timed region.

Prints one JSON line.  Besides the FP32 headline it carries the BF16 and FP16 storage runs (one
complete run each, with their relative L2 distance from the FP32-storage run and the 1e-2 storage
gate), the HBM ceiling of a hand-written streaming copy (chf_stream_copy, 4 GiB), and the FP64
CPU oracle timed on a bounded sample.  ``--workload single-shower`` measures the 256x256x2048,
4000-step configuration the same way (160-step slices), with errors against the stored FP64
oracle waveforms.

Counter summaries: ``--copy-probe`` adds a 256 MiB device copy before the runs (the
calibration dispatch for FETCH_SIZE / WRITE_SIZE); ``--summarize-pmc FETCH.csv WRITE.csv``
turns two rocprofv3 --pmc runs of that command into HBM bytes per launch of the sweep.

``--workload rz-8192`` (or rz-N) measures the paper's own axisymmetric (r, z) scheme instead:
a bench step is one full run of the N x N lattice (1 cm cells, Mur walls, the moving shower,
64 observers, N Yee steps) from zero fields.  ``--leg adjoint|batch|rz`` prints the
differentiation, 32-shower batch or (r, z) summary alone.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
COPY_PROBE_BYTES = 256 << 20
FUSED_KERNEL = "chf::k_fused<"
STEP2_KERNEL = "chf::k_step2<"
# the profiler leaves names it cannot demangle (the _Float16 instances) mangled
MANGLED = {FUSED_KERNEL: "_ZN3chf7k_fusedI", STEP2_KERNEL: "_ZN3chf7k_step2I"}
RZ_KERNEL = "k_rz_step2<"
RZ_BYTES_PER_NODE = 24.0  # read E_r, E_z, H_phi once and write them once (FP32)
FP64_VECTOR_PEAK_TFLOPS = 78.6
DFT_FLOPS_PER_TERM = 10.0  # 2 FMA into the sums + one complex rotation of the phase (4 mul, 2 add)
DTYPE = {"fp32": "f32", "bf16": "f32 (bf16 storage)", "fp16": "f32 (f16 storage)",
         "bf16x": "f32 (bf16 + 8-bit extension storage)"}
SLICES_PER_RUN = 25          # a bench step is one slice of a full run
STORAGE_GATE = 1e-2          # relative L2 the 16-bit storage runs must meet
COPY_CEILING_BYTES = 4 << 30  # source size of the streaming-copy ceiling probe


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_digest(files=("chf_kernels.hip", "chf_internal.h")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1001_5341_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def is_rz(workload: str) -> bool:
    return workload.startswith("rz-")


def kernel_digest_for(workload: str) -> str:
    return kernel_source_digest(("chf_rz.hip",) if is_rz(workload)
                                else ("chf_kernels.hip", "chf_step2.hip", "chf_cell.h", "chf_internal.h"))


def canonical_workload(name: str) -> str:
    """The full name of a workload given by its short name ("precision" ->
    "precision-512x512x4096"); (r, z) names and full names pass through."""
    if is_rz(name):
        return name
    from paper_1001_5341_amd import workloads as W

    try:
        return W.workload_by_name(name).name
    except KeyError:
        return name


def traffic_path(workload: str, storage: str) -> str:
    kern = "rz_step" if is_rz(workload) else "fused_sweep"
    return os.path.join(ROOT, "profiles", f"traffic_{kern}_{canonical_workload(workload)}_{storage}.json")


def measured_traffic(workload: str, storage: str, tile=None):
    """HBM bytes per launch of the dominant kernel from the committed counter summary, if it
    was taken on the current kernel source and (when given) the same tile shape; else None."""
    path = traffic_path(workload, storage)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_digest") != kernel_digest_for(workload):
        return None
    if tile is not None and rec.get("tile") != list(tile):
        return None
    return rec.get("bytes_per_launch")


def _dispatches(path: str, counter: str):
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                yield r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])


def summarize_pmc(fetch_csv: str, write_csv: str, workload: str, storage: str, command: str, tile=None):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the fused sweep, each scaled by what the
    same counter reads for the 256 MiB calibration copy (read 256 MiB, write 256 MiB)."""
    out = {}
    kname = RZ_KERNEL if is_rz(workload) else (STEP2_KERNEL if tile and tile[-1] == "fused2" else FUSED_KERNEL)
    for name, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = list(_dispatches(path, counter))
        copies = [v for k, g, v in rows if "copyBuffer" in k]
        if not copies:
            raise SystemExit(f"{path}: no calibration copy dispatch (run with --copy-probe)")
        copy_kib = max(copies)  # the 256 MiB probe is by far the largest copy
        fused = [v for k, g, v in rows if kname in k or (kname in MANGLED and k.startswith(MANGLED[kname]))]
        if not fused:
            raise SystemExit(f"{path}: no {kname} dispatch")
        factor = (COPY_PROBE_BYTES / 1024.0) / copy_kib
        out[name] = {"copy_probe_kib": copy_kib, "scale": factor, "dispatches": len(fused),
                     "raw_kib_per_launch": float(np.mean(fused)),
                     "bytes_per_launch": float(np.mean(fused)) * 1024.0 * factor}
    kdesc = ("axisymmetric two-step launch (k_rz_step2)" if is_rz(workload)
             else "two-step interior sweep (chf::k_step2)" if kname == STEP2_KERNEL
             else "fused interior sweep (chf::k_fused)")
    rec = {"workload": canonical_workload(workload), "storage": storage, "kernel": kdesc,
           "kernel_digest": kernel_digest_for(workload), "command": command, "tile": tile,
           "fetch": out["fetch"], "write": out["write"],
           "bytes_per_launch": out["fetch"]["bytes_per_launch"] + out["write"]["bytes_per_launch"]}
    path = traffic_path(workload, storage)
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec))


def cpu_baseline(w, n_steps: int = 300):
    """The FP64 oracle, as it stands, on a bounded sample of the workload: a 256x256x256 sub-grid
    (same spacing, medium, CPML and shower source; 8 observers placed inside it) for n_steps."""
    import oracle
    from paper_1001_5341_amd import workloads as W

    nz = 256
    sub = W.greisen_shower(w.seed, w.nx, w.ny, nz, n_steps, 8, zmax_frac=(0.4, 0.5),
                           length_range=(0.5, 1.0), r_range=(0.3, 1.0), name="cpu-sample")
    t0 = time.perf_counter()
    oracle.run(sub)
    dt = time.perf_counter() - t0
    rate = sub.n_cells * sub.n_steps / dt / 1e6
    cores = oracle.threads()
    # one thread, as the paper's sequential CPU code ran (a shorter sample of the same grid)
    one = sub.replace(n_steps=8)
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.run(one)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    return {"value": round(rate, 3), "unit": "Mcell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle on a {sub.nx}x{sub.ny}x{sub.nz} sub-grid of the workload "
                      f"(same medium, CPML-{sub.npml}, shower source, 8 observers), {sub.n_steps} steps, "
                      f"{dt:.1f} s",
            "value_1core": round(one.n_cells * one.n_steps / dt1 / 1e6, 3),
            "sample_1core": f"same sub-grid, {one.n_steps} steps on one thread, {dt1:.1f} s"}


def waveform_error(got: np.ndarray, ref: np.ndarray) -> dict:
    """Relative L2 per observer (3 components x all steps), max and median, and the largest
    peak-amplitude error."""
    err = np.sqrt(((got - ref) ** 2).sum(axis=(1, 2)) / (ref ** 2).sum(axis=(1, 2)))
    pk_ref = np.abs(ref).max(axis=(1, 2))
    pk = np.abs(np.abs(got).max(axis=(1, 2)) - pk_ref) / pk_ref
    return {"rel_l2_max": float(err.max()), "rel_l2_median": float(np.median(err)),
            "peak_amp_err_max": float(pk.max())}


def golden_error(key: str, w, got: np.ndarray):
    """Relative L2 (per observer, 3 components x all steps) and peak-amplitude error against
    the FP64 oracle's stored waveforms, when they exist for this exact workload."""
    from paper_1001_5341_amd.workloads import workload_digest

    gold = os.path.join(ROOT, "tests", "golden", f"{key}_oracle.npz")
    if not os.path.exists(gold):
        return None
    z = np.load(gold)
    if str(z["digest"]) != workload_digest(w):
        return None
    return waveform_error(got, z["waveforms"].astype(np.float64))


def slice_steps(w) -> int:
    if w.n_steps % SLICES_PER_RUN:
        raise SystemExit(f"{w.name}: {w.n_steps} Yee steps do not split into {SLICES_PER_RUN} slices")
    return w.n_steps // SLICES_PER_RUN


def timed_slices(plan, out, n_slices: int, s_len: int):
    """n_slices consecutive slices of s_len Yee steps from zero fields (zeroed before the timed
    region), each through chf_forward_timed; slice i covers steps (i mod 25) s_len onward, and a
    new run from zero fields starts after every 25th.  Returns (wall s, event s, summed
    fused-sweep ms, fused launches, waveforms of the first complete run or None)."""
    import torch

    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    fused_ms, first = 0.0, None
    plan.reset(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(n_slices):
        k = i % SLICES_PER_RUN
        if k == 0 and i > 0:
            plan.reset(stream)
        fused_ms += plan.forward_timed(s_len, out, k * s_len, stream)
        if k == SLICES_PER_RUN - 1 and first is None:
            first = out.clone()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, ev0.elapsed_time(ev1) / 1e3, fused_ms, n_slices * s_len, first


def copy_ceiling(n_bytes: int = COPY_CEILING_BYTES, reps: int = 5):
    """HBM bandwidth of the library's streaming copy (chf_stream_copy: 16-byte loads kept in flight
    per lane, non-temporal stores) over a few launch shapes; counts bytes read plus written."""
    import ctypes as ct

    import torch

    from paper_1001_5341_amd import _native as N

    L = N.lib()
    src = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    sh = ct.c_void_p(stream.cuda_stream)
    best, trials = None, []
    for u in (1, 2, 4, 8):
        for blocks in (1024, 2048, 4096, 8192):
            def go():
                N.check(L.chf_stream_copy(ct.c_void_p(dst.data_ptr()), ct.c_void_p(src.data_ptr()), n_bytes,
                                          u, blocks, sh), "chf_stream_copy")
            go()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            for _ in range(reps):
                go()
            ev1.record(stream)
            torch.cuda.synchronize()
            gbs = 2 * n_bytes * reps / (ev0.elapsed_time(ev1) / 1e3) / 1e9
            trials.append((u, blocks, round(gbs, 1)))
            if best is None or gbs > best[2]:
                best = (u, blocks, gbs)
    ok = bool(torch.equal(dst, src))
    del src, dst
    torch.cuda.empty_cache()
    return {"copy_ceiling_gbs": round(best[2], 1), "bytes_copied": n_bytes,
            "best_shape": {"loads_in_flight": best[0], "blocks": best[1], "threads_per_block": 256},
            "copy_verified": ok, "frac_of_peak": round(best[2] / HBM_PEAK_GBS, 4),
            "trials": [{"loads_in_flight": u, "blocks": b, "gbs": g} for u, b, g in trials]}


def roofline(info, fused_ms: float, yee_steps: int):
    """The dominant kernel (the interior sweep) from its hipEvent-timed launches: algorithmic
    bytes per launch / average launch duration.  A two-step launch advances two Yee steps and
    counts the one-step algorithmic bytes of both (temporal blocking: the figure can exceed what
    one pass could move, and the pass's own bytes are reported beside it)."""
    spl = int(info.get("steps_per_launch", 1) or 1)
    launches = yee_steps // spl
    alg = info["fused_cells"] * info["fused_bytes_per_cell"]
    avg_s = fused_ms / 1e3 / launches
    achieved = alg / avg_s / 1e9
    kdesc = ("chf::k_fused (fused H/E sweep of the interior rectangle, one launch per Yee step)" if spl == 1 else
             "chf::k_step2 (two Yee steps per pass over the interior rectangle: temporal blocking)")
    rec = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": kdesc,
           "launch_avg_us": round(avg_s * 1e6, 2), "launches": launches,
           "cells_per_launch": int(info["fused_cells"]),
           "bytes_per_cell": round(info["fused_bytes_per_cell"], 3),
           "alg_bytes_per_launch": int(alg)}
    if spl == 2:
        pass_gbs = info["fused_cells"] * info["pass_bytes_per_cell"] / avg_s / 1e9
        rec["temporal_blocking"] = {
            "steps_per_launch": 2, "pass_bytes_per_cell": round(info["pass_bytes_per_cell"], 3),
            "pass_achieved_gbs": round(pass_gbs, 1), "pass_frac": round(pass_gbs / HBM_PEAK_GBS, 4),
            "note": "achieved counts both steps at the one-step algorithmic bytes (single-step equivalent)"}
    return rec


def tile_shape(w, storage: str, args):
    """(waves, z_chunk, kernel): given on the command line, else from the autotuner (cached by
    shape; an explicit --kernel keeps its sweep kind with the tuned waves and z chunk)."""
    if args.waves or args.zchunk or args.kernel == "split" or args.no_tune:
        return args.waves, args.zchunk, args.kernel, False
    from paper_1001_5341_amd import autotune

    t = autotune.tune(w, storage)
    kernel = t["kernel"] if args.kernel == "auto" else args.kernel
    log(f"{storage}: tuned tile waves={t['waves']} z_chunk={t['z_chunk']} kernel={t['kernel']} "
        f"({'cached' if t['cached'] else 'measured'}, {t['ms_per_step']:.3f} ms/step)")
    return t["waves"], t["z_chunk"], kernel, True


def kernel_name(info) -> str:
    return {3: "fused_prefetch", 4: "fused2"}.get(info["kernel"], "fused")


def run_variant(w, storage: str, args, n_slices: int, warmup: int, dynamic: bool = False):
    import torch

    from paper_1001_5341_amd import solver

    waves, zchunk, kernel, tuned = tile_shape(w, storage, args)
    plan = solver.Plan(w, storage=storage, kernel=kernel, rows=args.rows, waves=waves,
                       zchunk=zchunk, device=torch.device("cuda:0"), dynamic_scaling=dynamic)
    info = plan.info()
    out = plan.new_waveforms()
    s_len = slice_steps(w)
    plan.reset()
    for i in range(warmup):
        plan.forward(s_len, out, (i % SLICES_PER_RUN) * s_len)
    torch.cuda.synchronize()
    if warmup:
        log(f"{storage}: {warmup} warm-up slices done")
    wall, ev_s, fused_ms, launches, full = timed_slices(plan, out, n_slices, s_len)
    spl = int(info.get("steps_per_launch", 1) or 1)
    log(f"{storage}: {n_slices} timed slices of {s_len} Yee steps, wall {wall:.3f} s, events {ev_s:.3f} s, "
        f"interior sweep {fused_ms / (launches // spl) * 1e3:.1f} us/launch ({spl} step(s) per launch)")
    got = full.cpu().numpy() if full is not None else None
    plan.close()
    info["tuned"] = tuned
    return info, wall, ev_s, fused_ms, launches, got


def rz_cpu_baseline(w, n_steps: int = 4):
    """The axisymmetric FP64 oracle (NumPy, one thread), as it stands, on the workload's own
    lattice for a few Yee steps from zero fields (its cost per step does not depend on the
    field values)."""
    from oracle import rz_oracle as R

    st = R.RZState(w)
    t0 = time.perf_counter()
    for _ in range(n_steps):
        st.step()
    dt = time.perf_counter() - t0
    return {"value": round(w.nr * w.nz * n_steps / dt / 1e6, 3), "unit": "Mcell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"NumPy FP64 oracle of the (r, z) scheme on the full {w.nr}x{w.nz} lattice, "
                      f"{n_steps} steps, {dt:.1f} s"}


def rz_measure(w, n_runs: int, warmup: int, vx=0, waves=0, zchunk=0, spl=0, storage="fp32", dynamic=False):
    """n_runs full runs through chf_rz_forward_timed; returns (info, wall s, event s,
    summed step-kernel ms, launches, waveforms)."""
    import torch

    from paper_1001_5341_amd import solver

    plan = solver.RZPlan(w, vx=vx, waves=waves, zchunk=zchunk, steps_per_launch=spl, storage=storage,
                         dynamic_scaling=dynamic, device=torch.device("cuda:0"))
    info = plan.info()
    out = plan.new_waveforms()
    for i in range(warmup):
        plan.run(out=out)
        log(f"rz warmup {i} done")
    wall, ev_s, ms, _ = timed_runs(plan, out, n_runs)
    spl = info["steps_per_launch"]
    launches = n_runs * (w.n_steps // spl + w.n_steps % spl)
    got = out.cpu().numpy()
    plan.close()
    return info, wall, ev_s, ms, launches, got


def rz_roofline(w, ms: float, launches: int, spl: int):
    """Algorithmic bytes of one launch: every marched node's E_r, E_z, H_phi read once and written
    once (24 B in FP32), whether the launch advances one Yee step or two; `effective` counts the
    bytes the same steps would move one step per pass."""
    nodes = w.nr * (w.nz - 1)  # rows 0..nz-2 are marched over every radial node
    alg = nodes * RZ_BYTES_PER_NODE
    avg_s = ms / 1e3 / launches
    achieved = alg / avg_s / 1e9
    name = ("k_rz_step2 (two Yee steps per launch: H, E_r, E_z, source and walls of both, the intermediate "
            "level in registers, and the previous launch's sampling)" if spl == 2 else
            "k_rz_step (H, E_r, E_z, source, walls and the previous step's sampling; one launch per Yee step)")
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": name, "steps_per_launch": spl,
            "launch_avg_us": round(avg_s * 1e6, 2), "launches": launches, "nodes_per_launch": nodes,
            "bytes_per_node": RZ_BYTES_PER_NODE, "alg_bytes_per_launch": int(alg),
            "effective_single_step_gbs": round(achieved * spl, 1),
            "effective_frac": round(achieved * spl / HBM_PEAK_GBS, 4)}


def rz_main(args):
    import torch

    from paper_1001_5341_amd import workloads as W

    w = W.rz_workload_by_name(args.workload)
    if args.time_steps:
        w = w.replace(n_steps=args.time_steps)
    torch.cuda.set_device(0)
    log(f"workload {w.name}: {w.nr}x{w.nz}, {w.n_steps} steps")
    if args.copy_probe:
        a = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    shape, tuned = (args.vx, args.waves, args.zchunk, args.steps_per_launch), False
    if not (args.no_tune or any(shape)):
        from paper_1001_5341_amd import autotune

        t = autotune.tune_rz(w)
        shape, tuned = tuple(t["shape"]), True
        log(f"rz: tuned shape (vx, waves, z_chunk, steps/launch) = {shape} "
            f"({'cached' if t['cached'] else 'measured'}, {t['ms_per_step']:.4f} ms/step)")
    info, wall, ev_s, ms, launches, got = rz_measure(w, args.steps, args.warmup, *shape)
    log(f"rz: {args.steps} timed runs, wall {wall:.3f} s, step kernel {ms / launches * 1e3:.1f} us/launch")
    roof = rz_roofline(w, ms, launches, info["steps_per_launch"])
    tile = [info["vx"], info["waves_per_block"], info["z_chunk"], info["steps_per_launch"]]
    roof["traffic"] = measured_traffic(args.workload, "fp32", tile) if not args.time_steps else None
    rec = {
        "metric": "Yee Mcell-updates/s and % HBM roofline of the axisymmetric (r, z) scheme, FP32",
        "value": round(w.nr * w.nz * w.n_steps * args.steps / wall / 1e6, 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded Greisen-like shower profile and observers; no datasets)",
        "config": {"workload": w.name, "grid_rz": [w.nr, w.nz], "yee_steps_per_run": w.n_steps,
                   "boundary": w.bc, "observers": w.n_obs,
                   "tile": {"vx": info["vx"], "waves_per_block": info["waves_per_block"],
                            "z_chunk": info["z_chunk"], "steps_per_launch": info["steps_per_launch"],
                            "autotuned": tuned},
                   "parallelism": "single GPU"},
        "roofline": roof,
        "waveforms_finite": bool(np.isfinite(got).all()),
    }
    if not args.time_steps and not args.no_variants:
        variants = {}
        for st, dyn in (("bf16", False), ("fp16", False), ("fp16", True)):
            name = st + ("-dynamic" if dyn else "")
            log(f"rz storage variant {name}")
            vinfo, vwall, _, vms, vl, vgot = rz_measure(w, 1, 0, *shape, storage=st, dynamic=dyn)
            vroof = rz_roofline(w, vms, vl, vinfo["steps_per_launch"])
            alg = w.nr * (w.nz - 1) * vinfo["bytes_per_cell_update"]
            variants[name] = {
                "value": round(w.nr * w.nz * w.n_steps / vwall / 1e6, 1), "unit": "Mcell-updates/s",
                "launch_avg_us": vroof["launch_avg_us"], "bytes_per_node": vinfo["bytes_per_cell_update"],
                "roofline_frac": round(alg / (vroof["launch_avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                "scale_e": vinfo["scale_e"], "scale_h": vinfo["scale_h"],
                "rel_l2_vs_fp32_run": float(np.linalg.norm(vgot - got) / np.linalg.norm(got)),
                "finite": bool(np.isfinite(vgot).all())}
        rec["storage_variants"] = variants
    if not args.time_steps:
        log("spectral post-processing of the run's waveforms")
        rec["spectral"] = spectral_measure(w, got)
    if not args.no_cpu_baseline:
        log("timing the (r, z) oracle on the host")
        rec["cpu_baseline"] = rz_cpu_baseline(w)
    print(json.dumps(rec), flush=True)


def spectral_measure(w, waves, n_freq: int = 1024, reps: int = 5):
    """FP64 DFT of the run's waveforms (all observers, both components) at n_freq frequencies up to
    2 GHz, then the theta projection and the far-field formula for the same observers."""
    import torch

    from paper_1001_5341_amd import spectral

    wt = torch.as_tensor(waves, device="cuda")
    om = 2 * np.pi * np.linspace(0.0, 2e9, n_freq)
    spectral.spectrum(wt, w.dt, om)  # warm-up
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        spec = spectral.spectrum(wt, w.dt, om)
    ev1.record()
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) / reps * 1e3
    n_series, n_t = wt.shape[0] * wt.shape[1], wt.shape[2]
    flops = DFT_FLOPS_PER_TERM * n_series * n_t * n_freq
    rt, wts = spectral.geometry(w)
    e_th, mag = spectral.project(spec, wts)
    ff = spectral.far_field(w, rt, om)
    torch.cuda.synchronize()
    ach = flops / (us * 1e-6) / 1e12
    return {"kernel": "k_spectrum (FP64 DFT, LDS-staged samples, re-anchored phase recurrence)",
            "series": n_series, "samples": n_t, "frequencies": n_freq, "launch_avg_us": round(us, 2),
            "roofline": {"bound": "alu", "achieved": round(ach, 2), "peak": FP64_VECTOR_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(ach / FP64_VECTOR_PEAK_TFLOPS, 4),
                         "flops_per_term": DFT_FLOPS_PER_TERM},
            "finite": bool(torch.isfinite(mag).all() and torch.isfinite(ff).all())}


# HBM bytes per node of one reverse step (FP32, outside the CPML slabs): sweep A reads Eb and Hb
# and writes Hb' (36 B), sweep B reads Hb' and Eb and writes Eb' (36 B); the neighbour terms are
# recomputed or exchanged on chip
ADJ_BYTES_PER_CELL = 72.0


def adjoint_summary():
    """Differentiation configuration (128x128x1024 CPML-10, 3000 steps, 16 observers, 128 profile
    bins, L = |w(q) - w(q*)|^2): forward run, one-sweep discrete adjoint, and the checkpointed
    gradient (forward with snapshots every 55 steps, then segment-wise recomputation and reverse
    steps), each timed once after a warm-up."""
    import torch

    from paper_1001_5341_amd import autotune, solver
    from paper_1001_5341_amd import workloads as W

    from paper_1001_5341_amd.workloads import workload_digest

    w, q_target = W.adjoint_problem()
    dev = torch.device("cuda:0")
    plan = autotune.tuned_plan(w, "fp32", device=dev)
    gold = os.path.join(ROOT, "tests", "golden", "adjoint_oracle.npz")
    z = np.load(gold) if os.path.exists(gold) else None
    if z is not None and str(z["digest"]) != workload_digest(w):
        z = None
    try:
        target = plan.run(q_bins=torch.from_numpy(q_target).to(dev))
        if z is not None:  # the FP64 oracle's target waveforms, so that dL/dq is comparable
            target = torch.from_numpy(z["w_star"].astype(np.float64)).to(dev)
        g = (2.0 * (plan.run() - target)).contiguous()

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            return out, time.perf_counter() - t0

        _, t_fwd = timed(lambda: plan.run())
        dq, t_adj = timed(lambda: plan.adjoint(g))
        dq_ck, t_ck = timed(lambda: solver.checkpointed_adjoint(plan, g, every=55, verify=False))
        same = bool(torch.equal(dq, dq_ck))
        finite = bool(torch.isfinite(dq).all())
        # permittivity map gradient: the same schedule, forward E levels kept per segment (run once)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gmap, dq_eps = solver.eps_sensitivity(plan, g, every=55)
        torch.cuda.synchronize()
        t_eps = time.perf_counter() - t0
        same_eps = bool(torch.equal(dq, dq_eps))
        del gmap
    finally:
        plan.close()
    cells = w.nx * w.ny * w.nz
    rate = cells * w.n_steps / t_adj
    acc = None
    if z is not None:
        ref = z["dl_dq"]
        acc = {"dl_dq_rel_l2": float(np.linalg.norm(dq.cpu().numpy() - ref) / np.linalg.norm(ref))}
    return {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "yee_steps": w.n_steps, "observers": w.n_obs,
            "bins": len(w.q_bins), "forward_ms": round(t_fwd * 1e3, 1), "adjoint_ms": round(t_adj * 1e3, 1),
            "checkpointed_gradient_ms": round(t_ck * 1e3, 1), "checkpoint_every": 55,
            "adjoint_value": round(rate / 1e6, 1), "unit": "Mcell-updates/s (reverse steps)",
            "adjoint_bytes_per_cell": ADJ_BYTES_PER_CELL,
            "adjoint_achieved_gbs": round(rate * ADJ_BYTES_PER_CELL / 1e9, 1),
            "adjoint_frac": round(rate * ADJ_BYTES_PER_CELL / 1e9 / HBM_PEAK_GBS, 4),
            "checkpointed_equals_one_sweep": same, "gradient_finite": finite,
            "eps_sensitivity_ms": round(t_eps * 1e3, 1), "eps_sensitivity_dq_equals_one_sweep": same_eps,
            "accuracy_vs_fp64_oracle": acc}


# batch members are tuned over the plain fused sweep of 7 or 8 rows: batched members that load a
# plane ahead ran slower (12.4 against 10.0 ms per step over the 32 members, same bits)
BATCH_CANDIDATES = tuple((wv, z, "fused") for wv in (7, 8) for z in (8, 12, 16, 24))


def batch_accuracy(ws, outs):
    """Waveform error of the members whose FP64 oracle waveforms are stored (all 32 of the
    batch), max over those members."""
    from paper_1001_5341_amd.workloads import workload_digest

    gold = os.path.join(ROOT, "tests", "golden", "batch_oracle.npz")
    if not os.path.exists(gold):
        return None
    z = np.load(gold)
    res = []
    for m in [int(v) for v in z["members"]]:
        if str(z[f"digest{m}"]) != workload_digest(ws[m]):
            return None
        res.append(waveform_error(outs[m].cpu().numpy(), z[f"member{m}"].astype(np.float64)))
    return {"members": [int(v) for v in z["members"]],
            "rel_l2_max": max(r["rel_l2_max"] for r in res),
            "peak_amp_err_max": max(r["peak_amp_err_max"] for r in res)}


def batch_summary():
    """Batched configuration: 32 showers of uneven grids (96^3 ... 256x256x1024, CPML-10, 16
    observers each, 2000 steps) advanced together in one hipGraph per run (chf_batch_run), with
    autotuned tile shapes (one waves_per_block for all members, z chunk per member).  One warm-up
    run (it also captures the graph), then one timed run; then the same for the persistent
    cooperative launch (chf_batch_run_persistent), compared bit for bit."""
    import torch

    from paper_1001_5341_amd import autotune, solver
    from paper_1001_5341_amd import workloads as W

    ws = W.batch_showers()
    shapes = autotune.tune_batch(ws, "fp32", candidates=BATCH_CANDIDATES, steps=24)
    plans = [solver.Plan(w, kernel=s_["kernel"], waves=s_["waves"], zchunk=s_["z_chunk"], device=torch.device("cuda:0"))
             for w, s_ in zip(ws, shapes)]
    batch = solver.Batch(plans)
    try:
        outs = [p.new_waveforms() for p in plans]
        batch.run(outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.run(outs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        finite = all(bool(torch.isfinite(o).all()) for o in outs)
        alg = sum(p.info()["bytes_per_cell_update"] * w.n_cells for p, w in zip(plans, ws))
        acc = batch_accuracy(ws, outs)
        # the same run as one persistent cooperative launch (every tile through the general fused
        # sweep, grid barriers between phases): same bits, timed after one warm-up run
        pouts = [p.new_waveforms() for p in plans]
        batch.run(pouts, persistent=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.run(pouts, persistent=True)
        torch.cuda.synchronize()
        pwall = time.perf_counter() - t0
        same = all(bool(torch.equal(a, b)) for a, b in zip(pouts, outs))
    finally:
        batch.close()
        for p in plans:
            p.close()
    T = ws[0].n_steps
    cells = sum(w.n_cells for w in ws)
    return {"workload": f"batch-{len(ws)}-showers", "members": len(ws), "yee_steps": T,
            "cells_total": int(cells), "value": round(cells * T / wall / 1e6, 1), "unit": "Mcell-updates/s",
            "ms_per_run": round(wall * 1e3, 1), "waves_per_block": shapes[0]["waves"],
            "z_chunks": sorted({s_["z_chunk"] for s_ in shapes}),
            "whole_step_bytes_per_cell": round(alg / cells, 3),
            "achieved_gbs": round(alg * T / wall / 1e9, 1),
            "frac": round(alg * T / wall / 1e9 / HBM_PEAK_GBS, 4), "finite": finite,
            "accuracy_vs_fp64_oracle": acc,
            "persistent_launch": {"value": round(cells * T / pwall / 1e6, 1), "ms_per_run": round(pwall * 1e3, 1),
                                  "frac": round(alg * T / pwall / 1e9 / HBM_PEAK_GBS, 4),
                                  "bitwise_equal_to_graph": same}}


def rz_summary(n: int = 8192, n_steps: int = 2048):
    """Short measurement of the axisymmetric path for the default line."""
    from paper_1001_5341_amd import workloads as W

    w = W.rz_paper_grid(n, n_steps=n_steps)
    info, wall, ev_s, ms, launches, got = rz_measure(w, 1, 1)
    roof = rz_roofline(w, ms, launches, info["steps_per_launch"])
    return {"workload": w.name, "yee_steps": n_steps, "value": round(w.nr * w.nz * n_steps / wall / 1e6, 1),
            "unit": "Mcell-updates/s", "roofline_frac": roof["frac"], "achieved_gbs": roof["achieved"],
            "launch_avg_us": roof["launch_avg_us"], "steps_per_launch": info["steps_per_launch"],
            "effective_frac": roof["effective_frac"],
            "note": "python bench.py --workload rz-8192 gives the full line"}


def storage_variant(w, st: str, args, ref, n_slices: int, ref_label: str, dynamic: bool = False):
    """One storage variant over n_slices slices (a complete run at the default 25), its speed,
    roofline fraction and its distance from `ref` (the FP64 oracle's stored waveforms when they
    exist for this workload, else the FP32-storage run of the same build).  `dynamic`: FP16 with
    the storage scale picked per launch."""
    vinfo, vwall, _, vms, vl, vgot = run_variant(w, st, args, n_slices, 1, dynamic)
    cells = w.nx * w.ny * w.nz
    v = {"value": round(cells * vl / vwall / 1e6, 1), "unit": "Mcell-updates/s",
         "roofline_frac": roofline(vinfo, vms, vl)["frac"],
         "fused_launch_avg_us": roofline(vinfo, vms, vl)["launch_avg_us"],
         "fused_bytes_per_cell": round(vinfo["fused_bytes_per_cell"], 3),
         "whole_step_bytes_per_cell": round(vinfo["bytes_per_cell_update"], 3),
         "scale_e": vinfo["scale_e"], "scale_h": vinfo["scale_h"],
         "dynamic_scaling": bool(vinfo.get("dynamic_scaling", 0)),
         "tile": {"vx": vinfo["vx"], "waves_per_block": vinfo["waves_per_block"], "z_chunk": vinfo["z_chunk"],
                  "kernel": kernel_name(vinfo)}}
    if vgot is not None and ref is not None:
        e = waveform_error(vgot, ref)
        v[f"accuracy_vs_{ref_label}"] = e
        v["storage_gate"] = STORAGE_GATE
        v["gate_met"] = bool(e["rel_l2_max"] <= STORAGE_GATE)
    return v


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=SLICES_PER_RUN,
                    help=f"timed slices ({SLICES_PER_RUN} slices = one complete run)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed slices before the timed region")
    ap.add_argument("--workload", default="precision")
    ap.add_argument("--storage", default="fp32", choices=["fp32", "bf16", "fp16", "bf16x"])
    ap.add_argument("--kernel", default="auto", choices=["auto", "fused", "fused_prefetch", "fused2", "split"])
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--vx", type=int, default=0, help="(r, z) path: radial nodes per lane")
    ap.add_argument("--steps-per-launch", type=int, default=0, help="(r, z) path: 1, or 2 (temporal blocking)")
    ap.add_argument("--time-steps", type=int, default=0, help="override the Yee steps per run (multiple of 25)")
    ap.add_argument("--no-tune", action="store_true", help="default tile shape instead of the autotuner's")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the BF16/FP16 storage runs")
    ap.add_argument("--no-copy-ceiling", action="store_true", help="skip the streaming-copy ceiling probe")
    ap.add_argument("--dynamic-fp16", action="store_true",
                    help="also run FP16 storage with the scale picked per launch (storage variant fp16_dynamic)")
    ap.add_argument("--legs", action="store_true",
                    help="also run the (r, z), differentiation and 32-shower batch summaries")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 256 MiB device copy first (counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--pmc-command", default="", help="command recorded in the counter summary")
    ap.add_argument("--leg", choices=["adjoint", "batch", "rz"], default=None,
                    help="run one extra leg alone and print its JSON")
    args = ap.parse_args()
    # tile shapes measured on MI355X ship with the package; missing shapes are tuned and added
    os.environ.setdefault("CHFDTD_TUNE_CACHE", os.path.join(ROOT, "paper_1001_5341_amd", "tune_cache_gfx950.json"))

    if args.summarize_pmc:
        tile = ([args.vx, args.waves, args.zchunk, args.steps_per_launch] if is_rz(args.workload)
                else [args.waves, args.zchunk, args.kernel if args.kernel in ("fused_prefetch", "fused2") else "fused"])
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload, args.storage,
                      args.pmc_command, tile)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU z-slab decomposition is design-only)"}))
        sys.exit(2)
    if args.leg:
        import torch

        torch.cuda.set_device(0)
        legs = {"adjoint": adjoint_summary, "batch": batch_summary, "rz": rz_summary}
        print(json.dumps(legs[args.leg]()), flush=True)
        return

    if is_rz(args.workload):
        rz_main(args)
        return

    import torch

    from paper_1001_5341_amd import workloads as W

    w = W.workload_by_name(args.workload)
    if args.time_steps:
        w = w.replace(n_steps=args.time_steps)
    s_len = slice_steps(w)
    torch.cuda.set_device(0)
    log(f"workload {w.name}: {w.nx}x{w.ny}x{w.nz}, {w.n_steps} steps per run, slices of {s_len}, "
        f"storage {args.storage}")
    if args.copy_probe:
        a = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    ceiling = None
    if not args.no_copy_ceiling:
        ceiling = copy_ceiling()
        log(f"streaming-copy ceiling {ceiling['copy_ceiling_gbs']} GB/s ({ceiling['best_shape']})")

    info, wall, ev_s, fused_ms, launches, got = run_variant(w, args.storage, args, args.steps, args.warmup)
    cells = w.nx * w.ny * w.nz
    updates = cells * launches
    roof = roofline(info, fused_ms, launches)
    roof["traffic"] = (measured_traffic(args.workload, args.storage,
                                        [info["waves_per_block"], info["z_chunk"], kernel_name(info)])
                       if not args.time_steps else None)
    if ceiling is not None:
        roof["copy_ceiling_gbs"] = ceiling["copy_ceiling_gbs"]
        roof["frac_of_copy_ceiling"] = round(roof["achieved"] / ceiling["copy_ceiling_gbs"], 4)
    # whole Yee step (all kernels) against the whole-grid algorithmic bytes, for context
    step_s = ev_s / launches
    roof["whole_step"] = {"bytes_per_cell": round(info["bytes_per_cell_update"], 3),
                          "achieved": round(info["bytes_per_cell_update"] * cells / step_s / 1e9, 1),
                          "frac": round(info["bytes_per_cell_update"] * cells / step_s / 1e9 / HBM_PEAK_GBS, 4),
                          "us_per_yee_step": round(step_s * 1e6, 2)}
    rec = {
        "metric": "Yee Mcell-updates/s and % HBM roofline, FP32 vs BF16-storage at stated L2 error",
        "value": round(updates / wall / 1e6, 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.storage],
        "data": "synthetic (seeded Greisen-like shower profile and observers; no datasets)",
        "config": {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "yee_steps_per_run": w.n_steps,
                   "yee_steps_per_bench_step": s_len,
                   "boundary": f"{w.bc}{w.npml}", "observers": w.n_obs, "storage": args.storage,
                   "kernel": {1: "split H/E sweeps", 2: "fused sweep (interior + boundary tiles)",
                              3: "fused sweep, interior tiles loading a plane ahead (+ boundary tiles)",
                              4: "two Yee steps per pass (temporal blocking; interior + boundary tiles)"}[info["kernel"]],
                   "tile": {"vx": info["vx"], "waves_per_block": info["waves_per_block"],
                            "z_chunk": info["z_chunk"], "autotuned": info["tuned"]},
                   "parallelism": "single GPU"},
        "roofline": roof,
    }
    if ceiling is not None:
        rec["copy_probe"] = ceiling
    acc = golden_error(args.workload, w, got) if got is not None else None
    if acc is not None:
        rec["accuracy_vs_fp64_oracle"] = acc
    elif got is not None:
        rec["accuracy_vs_fp64_oracle"] = None
        rec["accuracy_note"] = ("no stored FP64 oracle waveforms for this grid: the host oracle would need "
                                f"{cells * w.n_steps:.2e} cell-updates (about 54 GB and 15+ h on the host); "
                                "FP32 storage is checked against the oracle on the other configurations")
    if not args.no_variants and got is not None and args.storage == "fp32":
        ref, label = got, "fp32_run"
        gold = os.path.join(ROOT, "tests", "golden", f"{args.workload}_oracle.npz")
        if acc is not None and os.path.exists(gold):
            ref, label = np.load(gold)["waveforms"].astype(np.float64), "fp64_oracle"
        rec["storage_variants"] = {st: storage_variant(w, st, args, ref, SLICES_PER_RUN, label)
                                   for st in ("bf16", "bf16x", "fp16")}
        if args.dynamic_fp16:
            rec["storage_variants"]["fp16_dynamic"] = storage_variant(w, "fp16", args, ref, SLICES_PER_RUN, label,
                                                                      dynamic=True)
    if args.legs:
        log("axisymmetric (r, z) summary")
        rec["axisymmetric"] = rz_summary()
        log("adjoint and checkpointed gradient on the differentiation configuration")
        rec["adjoint"] = adjoint_summary()
        log("batch of 32 showers")
        rec["batch"] = batch_summary()
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a CPU sample")
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
