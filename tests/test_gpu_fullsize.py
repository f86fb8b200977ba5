"""Full-size parity, in the configuration the benchmark times (tile shape from the autotuner),
against FP64 oracle results stored by tests/golden/make_golden.py (which calls only the
oracle):

- single shower 256x256x2048, CPML-10, 4000 steps, 64 observers: every waveform;
- the 32-shower batch (uneven grids up to 256x256x1024, 2000 steps, 16 observers each), run
  as one batch: the sampled members the oracle can afford;
- differentiation 128x128x1024, 3000 steps, 128 profile bins: waveforms and dL/dq, by the
  one-sweep and the checkpointed (every 55 steps) adjoint.

The precision grid (512x512x4096) is beyond the oracle here (10 h and ~60 GB of host memory);
it is checked through properties that hold at any size: tile-shape and sweep-variant
invariance (bitwise) and the distance of BF16/FP16 storage from FP32 storage."""
import os

import numpy as np
import pytest
import torch

from paper_1001_5341_amd import autotune, solver
from paper_1001_5341_amd import workloads as W
from paper_1001_5341_amd.workloads import workload_digest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


def rel_l2(got, ref):
    return np.sqrt(((got - ref) ** 2).sum(axis=(1, 2)) / (ref ** 2).sum(axis=(1, 2)))


def stored(name):
    path = os.path.join(GOLD, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    return np.load(path)


def test_single_shower_full_size_against_stored_oracle(gpu):
    rec = stored("single-shower_oracle.npz")
    w = W.single_shower()
    assert str(rec["digest"]) == workload_digest(w), "stored waveforms belong to another workload"
    ref = rec["waveforms"].astype(np.float64)
    print(f"\n[gpu-fullsize] {w.name}: {w.n_cells * w.n_steps:.3e} cell-updates", flush=True)
    plan = autotune.tuned_plan(w, "fp32")
    got = plan.run(out=plan.new_waveforms(), graph=True).cpu().numpy()
    plan.close()
    err = rel_l2(got, ref)
    print("rel L2 max", err.max(), "median", np.median(err), flush=True)
    assert np.all(err <= 1e-5), err


def test_batch_full_size_sampled_members_against_stored_oracle(gpu):
    rec = stored("batch_oracle.npz")
    ws = W.batch_showers()
    members = [int(m) for m in rec["members"]]
    for m in members:
        assert str(rec[f"digest{m}"]) == workload_digest(ws[m])
    print(f"\n[gpu-fullsize] batch of {len(ws)}: "
          f"{sum(w.n_cells * w.n_steps for w in ws):.3e} cell-updates", flush=True)
    shapes = autotune.tune_batch(ws, "fp32")
    plans = [solver.Plan(w, kernel=s["kernel"], waves=s["waves"], zchunk=s["z_chunk"]) for w, s in zip(ws, shapes)]
    batch = solver.Batch(plans)
    outs = batch.run()
    for m in members:
        err = rel_l2(outs[m].cpu().numpy(), rec[f"member{m}"].astype(np.float64))
        print(ws[m].name, "rel L2 max", err.max(), flush=True)
        assert np.all(err <= 1e-5), (m, err)
    batch.close()
    for p in plans:
        p.close()


def test_adjoint_full_size_against_stored_oracle(gpu):
    rec = stored("adjoint_oracle.npz")
    w, q_target = W.adjoint_problem()
    assert str(rec["digest"]) == workload_digest(w)
    print(f"\n[gpu-fullsize] {w.name}: forward + adjoint", flush=True)
    plan = autotune.tuned_plan(w, "fp32")
    w_q = plan.run()
    err = rel_l2(w_q.cpu().numpy(), rec["w_q"].astype(np.float64))
    print("waveforms rel L2 max", err.max(), flush=True)
    assert np.all(err <= 1e-5), err
    w_star = torch.from_numpy(rec["w_star"].astype(np.float64)).to(w_q.device)
    dl_dw = 2.0 * (w_q - w_star)
    grad = plan.adjoint(dl_dw)
    plan.sync()
    # the checkpointed schedule (a snapshot every 55 steps, segments recomputed in reverse)
    # gives the same bits
    grad_ck = solver.checkpointed_adjoint(plan, dl_dw, every=55)
    plan.close()
    assert torch.equal(grad_ck, grad)
    grad = grad.cpu().numpy()
    ref = rec["dl_dq"]
    gerr = np.linalg.norm(grad - ref) / np.linalg.norm(ref)
    print("dL/dq rel L2", gerr, flush=True)
    assert gerr <= 1e-4, gerr


def test_precision_grid_full_size_invariants(gpu):
    """512x512x4096 (the precision workload's grid, shower and observers) for 400 steps: the
    fused sweep with two tile shapes and the split sweeps give identical fields; FP16 storage
    stays within the 1e-2 gate of FP32 storage, and BF16 within its error envelope (1e-1, a
    regression bound: BF16 misses the gate)."""
    w = W.precision_shower().replace(n_steps=400)
    print(f"\n[gpu-fullsize] {w.name} x {w.n_steps} steps", flush=True)

    def ez_after(**kw):
        plan = solver.Plan(w, **kw)
        plan.run()
        ez = plan.get_field(2)
        plan.close()
        del plan
        torch.cuda.empty_cache()
        return ez

    base = ez_after(kernel="fused", zchunk=16)
    assert torch.count_nonzero(base).item() > 0
    assert torch.equal(ez_after(kernel="fused", zchunk=24), base)
    assert torch.equal(ez_after(kernel="split"), base)
    nb = torch.linalg.vector_norm(base.double())
    for storage, tol in (("fp16", 1e-2), ("bf16", 1e-1)):
        e = torch.linalg.vector_norm(ez_after(storage=storage).double() - base.double()) / nb
        print(storage, "Ez rel L2 vs FP32 storage", e.item(), flush=True)
        assert e.item() <= tol
