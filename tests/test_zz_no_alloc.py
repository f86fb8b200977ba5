"""chf_forward_scratch (the entry point that allocates nothing: its fields, CPML state and tables
live in the library's static device array) against chf_forward on a bound workspace, through the
C ABI: two calls in a row, the second on a smaller lattice, each bitwise equal to the same plan's
ordinary run.  Also: the plan's own workspace state is untouched by the scratch call, and a plan
larger than the array is refused before any device work."""
import ctypes as ct
import sys

import numpy as np
import pytest
import torch

from paper_1001_5341_amd import _native as N
from paper_1001_5341_amd import solver
from paper_1001_5341_amd import workloads as W


def banner(msg):
    print(f"\n[no-alloc] {msg}", flush=True)
    sys.stdout.flush()


def test_plan_above_scratch_size_is_refused():
    # host-side check: no device call happens before the size test
    w = W.small_shower(seed=3, nx=256, ny=256, nz=256, n_steps=4, n_obs=2, npml=8)
    h = solver.create_plan_handle(w)
    L = N.lib()
    try:
        nbytes = ct.c_uint64()
        N.check(L.chf_plan_workspace_bytes(h, ct.byref(nbytes)), "chf_plan_workspace_bytes")
        assert nbytes.value > L.chf_scratch_bytes()
        dummy = ct.c_void_p(256)  # never dereferenced: the call returns before touching it
        st = L.chf_forward_scratch(h, ct.c_void_p(), ct.c_void_p(), dummy)
        assert N.STATUS[st] == "CHF_ENOMEM"
        assert b"static scratch" in L.chf_last_error()
    finally:
        L.chf_plan_destroy(h)


@pytest.mark.gpu
def test_scratch_forward_matches_bound_workspace(gpu):
    L = N.lib()
    cap = L.chf_scratch_bytes()
    cases = [
        ("first", W.small_shower(seed=11, nx=72, ny=60, nz=150, n_steps=200, n_obs=6, npml=8), "fp32"),
        ("second, smaller", W.small_shower(seed=12, nx=40, ny=36, nz=64, n_steps=90, n_obs=3, npml=5), "fp16"),
    ]
    for label, w, storage in cases:
        plan = solver.Plan(w, storage=storage, device=gpu)
        assert plan.workspace_bytes <= cap, (plan.workspace_bytes, cap)
        banner(f"{label}: {w.nx}x{w.ny}x{w.nz}, {w.n_steps} steps, {storage}, "
               f"workspace {plan.workspace_bytes} of {cap} bytes")
        ref = plan.run().cpu().numpy()
        ez_before = plan.get_field(2).cpu().numpy()
        got = plan.run_scratch().cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(got, ref), float(np.abs(got - ref).max())
        assert np.abs(ref).max() > 0  # the source reached the observers
        # the plan's own workspace still holds its own run's final state
        assert np.array_equal(plan.get_field(2).cpu().numpy(), ez_before)
        plan.close()
