"""Full-size parity: the single-shower workload (256x256x2048 cells, CPML-10, 4000 steps,
64 observers) on the GPU, in the configuration the benchmark times, against the FP64 oracle's
waveforms stored by tests/golden/make_golden.py (which calls only the oracle)."""
import os

import numpy as np
import pytest

from paper_1001_5341_amd import solver
from paper_1001_5341_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "single-shower_oracle.npz")


def test_single_shower_full_size_against_stored_oracle(gpu):
    from paper_1001_5341_amd.workloads import workload_digest

    if not os.path.exists(GOLD):
        pytest.skip("stored oracle waveforms not generated")
    rec = np.load(GOLD)
    w = W.single_shower()
    assert str(rec["digest"]) == workload_digest(w), "stored waveforms belong to another workload"
    ref = rec["waveforms"].astype(np.float64)
    print(f"\n[gpu-fullsize] {w.name}: {w.n_cells * w.n_steps:.3e} cell-updates", flush=True)
    plan = solver.Plan(w)
    got = plan.run(out=plan.new_waveforms(), graph=True).cpu().numpy()
    plan.close()
    err = np.sqrt(((got - ref) ** 2).sum(axis=(1, 2)) / (ref ** 2).sum(axis=(1, 2)))
    print("rel L2 max", err.max(), "median", np.median(err), flush=True)
    assert np.all(err <= 1e-5), err
