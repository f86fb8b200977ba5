"""Tile-shape autotuner: every candidate reproduces the same waveforms bit for bit, the fastest
is cached by shape, and a tuned plan still matches the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1001_5341_amd import autotune
from paper_1001_5341_amd import workloads as W

pytestmark = pytest.mark.gpu

CANDS = [(4, 8, "fused"), (8, 16, "fused"), (4, 150, "fused"), (8, 5, "fused"),
         (8, 16, "fused_prefetch"), (7, 9, "fused_prefetch")]


def test_autotune_verifies_caches_and_matches_oracle(gpu, tmp_path):
    w = W.small_shower()
    path = str(tmp_path / "tune.json")
    print(f"\n[gpu-autotune] {w.name}", flush=True)
    first = autotune.tune(w, "fp32", steps=40, cache_path=path, candidates=CANDS)
    assert not first["cached"]
    timed = [t for t in first["trials"] if "ms_per_step" in t]
    assert len(timed) == len(CANDS) and all(t["bitwise_equal"] for t in timed)
    best = (first["waves"], first["z_chunk"], first["kernel"])
    assert best in CANDS
    again = autotune.tune(w, "fp32", steps=40, cache_path=path, candidates=CANDS)
    assert again["cached"] and (again["waves"], again["z_chunk"], again["kernel"]) == best
    plan = autotune.tuned_plan(w, "fp32", cache_path=path, candidates=CANDS)
    got = plan.run().cpu().numpy()
    plan.close()
    ref = oracle.run(w)
    err = np.sqrt(((got - ref) ** 2).sum(axis=(1, 2)) / (ref ** 2).sum(axis=(1, 2)))
    assert np.all(err <= 1e-5), err


def test_rz_autotune_verifies_and_caches(tmp_path):
    """The (r, z) tuner times every shape, requires identical bits from all of them, caches the
    winner, and the tuned plan matches the oracle."""
    import numpy as np

    from oracle import rz_oracle
    from paper_1001_5341_amd import autotune, workloads as W

    w = W.rz_small(nr=200, nz=300, n_steps=400, n_obs=4)
    cache = str(tmp_path / "tune.json")
    cands = [(4, 1, 64, 2), (8, 2, 32, 2), (4, 4, 16, 1), (2, 2, 8, 1)]
    t = autotune.tune_rz(w, steps=40, cache_path=cache, candidates=cands)
    assert not t["cached"] and all(x.get("bitwise_equal") for x in t["trials"])
    assert autotune.tune_rz(w, steps=40, cache_path=cache, candidates=cands)["cached"]
    plan = autotune.tuned_rz_plan(w, cache_path=cache, candidates=cands)
    try:
        got = plan.run().cpu().numpy()
    finally:
        plan.close()
    ref = rz_oracle.run(w)
    assert np.abs(ref).max() > 0
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5
