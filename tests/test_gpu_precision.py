"""Reduced-precision field storage (FP32 arithmetic, FP64 observer accumulation) against the FP64
oracle, relative L2 per observer.

The storage gate is 1e-2.  FP16 storage with power-of-two per-field scales meets it (~2e-3 here)
and is held to it: that is the parity claim for 16-bit storage.  BF16 storage (8-bit mantissa)
does not meet it: the rounding noise of every stored update accumulates along the propagation
path to ~1.6e-2 on this workload (5.9e-2 on the 256x256x2048 shower), and stochastic rounding
measured worse.  The BF16 test is therefore an error-envelope regression check (bound 2e-2,
about 1.25x the measured value), not a parity claim; the benchmark reports BF16 with
gate_met = false.  BF16X (BF16 with an 8-bit mantissa extension, 3 bytes per value) keeps 16
significant bits, 2^8 times BF16's precision, and is held to the gate (and, as a regression
check, to 1e-3)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1001_5341_amd import solver
from paper_1001_5341_amd import workloads as W

pytestmark = pytest.mark.gpu

GATE = 1e-2          # the storage gate (FP16 is held to it)
BF16_ENVELOPE = 2e-2  # BF16: regression bound on its measured error, not the gate


def rel_l2(got, ref):
    return np.sqrt(((got - ref) ** 2).sum(axis=(1, 2)) / (ref ** 2).sum(axis=(1, 2)))


@pytest.fixture(scope="module")
def shower():
    w = W.small_shower(seed=12, nx=64, ny=56, nz=120, n_steps=240, n_obs=6, npml=8)
    return w, oracle.run(w)


def _storage_error(shower, storage):
    w, ref = shower
    print(f"\n[gpu-precision] {storage}", flush=True)
    plan = solver.Plan(w, storage=storage)
    info = plan.info()
    got = plan.run().cpu().numpy()
    plan.close()
    err = rel_l2(got, ref)
    peak = np.abs(np.abs(got).max(axis=(1, 2)) - np.abs(ref).max(axis=(1, 2))) / np.abs(ref).max(axis=(1, 2))
    print(storage, "scales", info["scale_e"], info["scale_h"], "rel L2 max", err.max(),
          "median", np.median(err), "peak err max", peak.max())
    sys.stdout.flush()
    assert np.all(np.isfinite(got))
    return err


def test_fp16_storage_meets_the_gate(gpu, shower):
    err = _storage_error(shower, "fp16")
    assert np.all(err <= GATE), err


def test_bf16x_storage_meets_the_gate(gpu, shower):
    err = _storage_error(shower, "bf16x")
    assert np.all(err <= GATE), err
    assert np.all(err <= 1e-3), err  # 2^-8 of BF16's noise: far inside the gate


def test_bf16_storage_error_envelope(gpu, shower):
    """Regression check of BF16's error (it misses the 1e-2 gate; see the module docstring)."""
    err = _storage_error(shower, "bf16")
    assert err.max() > GATE / 10  # the measured error is of the expected size, not accidentally tiny
    assert np.all(err <= BF16_ENVELOPE), err


@pytest.mark.parametrize("storage", ["bf16", "fp16", "bf16x"])
def test_reduced_storage_fused_equals_split(gpu, shower, storage):
    w, _ = shower
    a = solver.Plan(w, storage=storage, kernel="fused")
    b = solver.Plan(w, storage=storage, kernel="split")
    ra = a.run().cpu().numpy()
    rb = b.run().cpu().numpy()
    a.close()
    b.close()
    assert np.array_equal(ra, rb)
