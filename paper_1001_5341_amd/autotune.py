"""Tile-shape autotuners (the 3-D fused sweep; the (r, z) step kernels), with a JSON cache.

For one workload shape it times every candidate (waves per workgroup x z chunk x sweep kind:
the plain fused sweep, or the one whose interior tiles issue their loads a plane ahead) over a
short run of the real step (interior and boundary sweeps, source, gather) and keeps the fastest.
The short run starts from pseudo-random fields, so every node is exercised from the first step,
and every candidate must reproduce the first candidate's observer waveforms and an exact digest
of all six final field components bit for bit: the per-node arithmetic is the same in every
tile shape, so a difference means a bug and the tuner raises instead of picking it.

Cache: a JSON object keyed by device architecture, storage type, boundary and grid shape,
stored at ``$CHFDTD_TUNE_CACHE`` or ``~/.cache/chfdtd/tune.json``.
"""
from __future__ import annotations

import json
import os
from typing import Iterable, Optional, Sequence, Tuple

import torch

from . import _native as N
from . import solver

# (waves per workgroup, z chunk, kernel); shapes a grid does not take are skipped: the prefetching
# sweep takes 4 or 5 rows on rows wider than 256 nodes (two waves per row) and 4-11 otherwise,
# the two-step sweep ("fused2") rows of at most 256 nodes with PEC or CPML walls
CANDIDATES: Tuple[Tuple[int, int, str], ...] = (
    tuple((w, z, "fused") for w in (4, 7, 8, 11, 15) for z in (8, 12, 16, 24, 32))
    + tuple((w, z, "fused_prefetch") for w in (4, 5, 7, 8, 11) for z in (8, 12, 16, 24, 32))
    + tuple((w, z, "fused2") for w in (7, 8) for z in (16, 24, 32)))


def _cand(c) -> Tuple[int, int, str]:
    c = tuple(c)
    return c if len(c) == 3 else (c[0], c[1], "fused")


def default_cache_path() -> str:
    return os.environ.get("CHFDTD_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "chfdtd", "tune.json"))


def shape_key(w, storage: str, device=None) -> str:
    arch = torch.cuda.get_device_properties(device or torch.cuda.current_device()).gcnArchName.split(":")[0]
    npml = w.npml if w.bc == "cpml" else 0
    return f"{arch}/{storage}/{w.bc}{npml}/{w.nx}x{w.ny}x{w.nz}"


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path: str, table: dict) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def field_digest(plan, stream=None) -> Tuple[int, ...]:
    """Exact digest of the current time level, one integer per component: the sum over nodes of
    (the FP32 bit pattern as an unsigned integer) x (node index mod 65521 + 1), modulo 2^64.  Two
    levels that differ in one value by d differ by d m mod 2^64 != 0 (|d m| < 2^48)."""
    out = []
    for c in range(6):
        bits = plan.get_field(c, stream).view(torch.int32).reshape(-1)
        acc = torch.zeros((), dtype=torch.int64, device=bits.device)
        step = 1 << 25
        for s in range(0, bits.numel(), step):
            seg = bits[s:s + step].to(torch.int64) & 0xFFFFFFFF
            mul = torch.arange(s, s + seg.numel(), dtype=torch.int64, device=bits.device) % 65521 + 1
            acc += (seg * mul).sum()  # int64 sums wrap modulo 2^64 in any order
        out.append(int(acc))
        del bits
    return tuple(out)


def _seed_fields(plan, stream=None):
    """Pseudo-random initial fields (the same for every candidate), stored values in [-1, 1), so
    that every node -- walls, layers, tile edges -- takes a non-trivial update from the first
    step; the source and the observers see them as any other field."""
    info = plan.info()
    w = plan.w
    g = torch.Generator(device=plan.device)
    g.manual_seed(20260301)
    for c in range(6):
        scale = info["scale_e"] if c < 3 else info["scale_h"]
        v = torch.rand((w.nz, w.ny, w.nx), generator=g, device=plan.device, dtype=torch.float32)
        plan.set_field(c, (v * 2 - 1) / scale, stream)
        del v


def _time_candidate(w, storage: str, waves: int, zchunk: int, steps: int, device, kernel: str = "fused"):
    """ms per step of one candidate, with its waveforms and final-field digest from random
    initial fields (each run twice: the two results must agree bit for bit)."""
    plan = solver.Plan(w.replace(n_steps=steps), storage=storage, kernel=kernel, waves=waves,
                       zchunk=zchunk, device=device)
    try:
        out = plan.new_waveforms()
        stream = torch.cuda.current_stream(device)
        plan.reset(stream)
        _seed_fields(plan, stream)
        plan.forward(steps, out, 0, stream=stream)  # warm-up, also the bitwise reference run
        ref = (out.clone(), field_digest(plan, stream))
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        plan.reset(stream)
        _seed_fields(plan, stream)
        out.zero_()
        ev0.record(stream)
        plan.forward(steps, out, 0, stream=stream)
        ev1.record(stream)
        plan.sync(stream)
        ms = ev0.elapsed_time(ev1) / steps
        got = (out, field_digest(plan, stream))
        if not (torch.equal(got[0], ref[0]) and got[1] == ref[1]):
            raise RuntimeError(f"tile shape waves={waves} z_chunk={zchunk} {kernel}: run-to-run results differ")
        if not bool(torch.isfinite(out).all()) or float(out.abs().max()) == 0.0:
            raise RuntimeError(f"tile shape waves={waves} z_chunk={zchunk} {kernel}: no finite, non-zero waveform "
                               "to compare")
        return ms, (out.cpu(), got[1]), plan.info()
    finally:
        plan.close()


def tune(w, storage: str = "fp32", steps: int = 48, cache_path: Optional[str] = None,
         candidates: Optional[Sequence[Tuple[int, int]]] = None, use_cache: bool = True,
         device=None, key_suffix: str = "") -> dict:
    """Best (waves_per_block, z_chunk, kernel) for this workload shape; cached by shape_key().
    A cache entry without a kernel is the plain fused sweep."""
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    path = cache_path or default_cache_path()
    key = shape_key(w, storage, device) + key_suffix
    cands = [_cand(c) for c in (candidates or CANDIDATES)]
    if use_cache:
        hit = _load(path).get(key)
        if hit and (hit["waves"], hit["z_chunk"], hit.get("kernel", "fused")) in cands:
            return dict(hit, kernel=hit.get("kernel", "fused"), cached=True)
    steps = max(2, min(steps, w.n_steps))
    trials, ref = [], None
    for waves, zchunk, kernel in cands:
        try:
            ms, wave, info = _time_candidate(w, storage, waves, zchunk, steps, device, kernel)
        except N.ChfError as exc:  # shape not valid for this grid (e.g. 8 waves on wide rows)
            trials.append({"waves": waves, "z_chunk": zchunk, "kernel": kernel, "error": exc.status})
            continue
        if ref is None:
            ref = wave
        elif not (torch.equal(wave[0], ref[0]) and wave[1] == ref[1]):
            raise RuntimeError(f"tile shape waves={waves} z_chunk={zchunk} {kernel} changes the results")
        trials.append({"waves": waves, "z_chunk": zchunk, "kernel": kernel, "ms_per_step": ms,
                       "vx": info["vx"], "bitwise_equal": True, "guard": "fields+waveforms"})
    timed = [t for t in trials if "ms_per_step" in t]
    if not timed:
        raise RuntimeError(f"no valid tile shape for {key}")
    best = min(timed, key=lambda t: t["ms_per_step"])
    rec = {"waves": best["waves"], "z_chunk": best["z_chunk"], "kernel": best["kernel"],
           "ms_per_step": best["ms_per_step"], "steps": steps, "trials": trials}
    table = _load(path)
    table[key] = rec
    _store(path, table)
    return dict(rec, cached=False)


def tuned_plan(w, storage: str = "fp32", **kw) -> "solver.Plan":
    """A Plan whose fused-sweep tile shape comes from tune()."""
    t = tune(w, storage, **kw)
    return solver.Plan(w, storage=storage, kernel=t["kernel"], waves=t["waves"], zchunk=t["z_chunk"],
                       device=kw.get("device"))


def tune_batch(workloads: Iterable, storage: str = "fp32", **kw) -> list:
    """Per-member z chunks for a batch, with one waves_per_block and one sweep kind for all
    members (a batch holds one of each): the most common best pair.  Cached under the member
    shape's key with the suffix "/batch", apart from the plan tunings of the same shape."""
    kw.setdefault("key_suffix", "/batch")
    res = [tune(w, storage, **kw) for w in workloads]
    pairs = [(r["waves"], r["kernel"]) for r in res]
    waves, kernel = max(sorted(set(pairs)), key=pairs.count)
    return [{"waves": waves, "z_chunk": r["z_chunk"], "kernel": kernel} for r in res]


# ------------------------------------------------------------------ axisymmetric (r, z) scheme
# (vx, waves per workgroup, z chunk, Yee steps per launch)
RZ_CANDIDATES: Tuple[Tuple[int, int, int, int], ...] = (
    (4, 1, 32, 2), (4, 1, 64, 2), (4, 2, 32, 2), (4, 2, 64, 2), (4, 4, 32, 2), (4, 4, 64, 2),
    (8, 1, 64, 2), (8, 2, 32, 2), (4, 4, 64, 1), (4, 1, 64, 1))


def rz_shape_key(w, device=None) -> str:
    arch = torch.cuda.get_device_properties(device or torch.cuda.current_device()).gcnArchName.split(":")[0]
    return f"{arch}/rz/{w.bc}/{w.nr}x{w.nz}"


def tune_rz(w, steps: int = 64, cache_path: Optional[str] = None,
            candidates: Optional[Sequence[Tuple[int, int, int, int]]] = None, use_cache: bool = True,
            device=None) -> dict:
    """Fastest (vx, waves, z_chunk, steps_per_launch) for an (r, z) lattice; every candidate must
    reproduce the first one's waveforms and final fields bit for bit."""
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    path = cache_path or default_cache_path()
    key = rz_shape_key(w, device)
    cands = [tuple(c) for c in (candidates or RZ_CANDIDATES)]
    if use_cache:
        hit = _load(path).get(key)
        if hit and tuple(hit["shape"]) in cands:
            return dict(hit, cached=True)
    steps = max(2, min(steps, w.n_steps))
    wt = w.replace(n_steps=steps)
    trials, ref = [], None
    for vx, waves, zc, spl in cands:
        try:
            plan = solver.RZPlan(wt, vx=vx, waves=waves, zchunk=zc, steps_per_launch=spl, device=device)
        except N.ChfError as exc:
            trials.append({"shape": [vx, waves, zc, spl], "error": exc.status})
            continue
        try:
            out = plan.new_waveforms()
            stream = torch.cuda.current_stream(device)
            plan.reset(stream)
            plan.forward(steps, out, 0, stream=stream)  # warm-up
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            out.zero_()
            plan.reset(stream)
            ev0.record(stream)
            plan.forward(steps, out, 0, stream=stream)
            ev1.record(stream)
            plan.sync(stream)
            ms = ev0.elapsed_time(ev1) / steps
            got = (out.cpu(), torch.stack([plan.get_field(c) for c in range(3)]).cpu())
        finally:
            plan.close()
        if ref is None:
            ref = got
        elif not (torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])):
            raise RuntimeError(f"(r, z) shape {(vx, waves, zc, spl)} changes the results")
        trials.append({"shape": [vx, waves, zc, spl], "ms_per_step": ms, "bitwise_equal": True})
    timed = [t for t in trials if "ms_per_step" in t]
    if not timed:
        raise RuntimeError(f"no valid (r, z) shape for {key}")
    best = min(timed, key=lambda t: t["ms_per_step"])
    rec = {"shape": best["shape"], "ms_per_step": best["ms_per_step"], "steps": steps, "trials": trials}
    table = _load(path)
    table[key] = rec
    _store(path, table)
    return dict(rec, cached=False)


def tuned_rz_plan(w, **kw) -> "solver.RZPlan":
    t = tune_rz(w, **kw)
    vx, waves, zc, spl = t["shape"]
    return solver.RZPlan(w, vx=vx, waves=waves, zchunk=zc, steps_per_launch=spl, device=kw.get("device"))
