"""Batched execution: showers of uneven grids advanced by one launch per phase per step (one
hipGraph for the run) give exactly the waveforms of each shower run alone."""
import numpy as np
import pytest

import oracle
from paper_1001_5341_amd import _native, solver
from paper_1001_5341_amd import workloads as W

pytestmark = pytest.mark.gpu


def members(steps=110):
    return [
        W.small_shower(seed=31, nx=40, ny=40, nz=64, n_steps=steps, n_obs=3, npml=6),
        W.small_shower(seed=32, nx=72, ny=60, nz=96, n_steps=steps, n_obs=4, npml=8),
        W.small_shower(seed=33, nx=130, ny=48, nz=80, n_steps=steps, n_obs=2, npml=6),
        W.small_shower(seed=34, nx=36, ny=44, nz=70, n_steps=steps, n_obs=3, bc="pec"),
        W.gaussian_cube(seed=35, n=32, n_steps=steps),  # Mur boundary
    ]


def test_batch_equals_single_runs(gpu):
    ws = members()
    print("\n[gpu-batch] singles", flush=True)
    singles = []
    for w in ws:
        p = solver.Plan(w)
        singles.append(p.run().cpu().numpy())
        p.close()
    print("[gpu-batch] batch", flush=True)
    plans = [solver.Plan(w) for w in ws]
    batch = solver.Batch(plans)
    for rep in range(2):
        outs = [o.cpu().numpy() for o in batch.run()]
        for a, b in zip(outs, singles):
            assert np.array_equal(a, b), rep
    batch.close()
    for p in plans:
        p.close()
    # plain 11-row tiles (12-wave workgroups) in the batched interior and boundary sweeps
    print("[gpu-batch] batch, 11-row tiles", flush=True)
    plans = [solver.Plan(w, kernel="fused", waves=11, zchunk=9) for w in ws]
    batch = solver.Batch(plans)
    outs = [o.cpu().numpy() for o in batch.run()]
    for a, b in zip(outs, singles):
        assert np.array_equal(a, b)
    batch.close()
    for p in plans:
        p.close()


def test_prefetching_batch_equals_single_runs(gpu):
    """Members whose tiles load a plane ahead (7-row tiles: the boundary tiles too; 11-row tiles)
    give the plain single runs' bits; a batch does not mix the two sweep kinds."""
    ws = members()
    singles = []
    for w in ws:
        p = solver.Plan(w, kernel="fused", waves=7)
        singles.append(p.run().cpu().numpy())
        p.close()
    for waves in (11, 7):  # 11 rows: 12-wave workgroups, plain boundary sweeps
        print(f"\n[gpu-batch] prefetching batch, {waves}-row tiles", flush=True)
        plans = [solver.Plan(w, kernel="fused_prefetch", waves=waves) for w in ws]
        batch = solver.Batch(plans)
        outs = [o.cpu().numpy() for o in batch.run()]
        for a, b in zip(outs, singles):
            assert np.array_equal(a, b)
        batch.close()
        if waves == 11:
            for p in plans:
                p.close()
    plain = solver.Plan(ws[0], kernel="fused", waves=7)
    with pytest.raises(_native.ChfError) as e:
        solver.Batch([plans[1], plain])
    assert e.value.status == "CHF_EINVAL"
    plain.close()
    for p in plans:
        p.close()


def test_batch_member_against_oracle(gpu):
    ws = members(steps=90)[:3]
    plans = [solver.Plan(w) for w in ws]
    batch = solver.Batch(plans)
    outs = batch.run()
    ref = oracle.run(ws[1])
    got = outs[1].cpu().numpy()
    err = np.sqrt(((got - ref) ** 2).sum(axis=(1, 2)) / (ref ** 2).sum(axis=(1, 2)))
    assert np.all(err <= 1e-5), err
    batch.close()


def test_batch_rejects_mismatched_steps(gpu):
    a = solver.Plan(W.small_shower(seed=1, nx=40, ny=40, nz=60, n_steps=10, n_obs=2, npml=6))
    b = solver.Plan(W.small_shower(seed=2, nx=40, ny=40, nz=60, n_steps=12, n_obs=2, npml=6))
    with pytest.raises(_native.ChfError) as e:
        solver.Batch([a, b])
    assert e.value.status == "CHF_EINVAL"


@pytest.mark.parametrize("waves", [7, 11])
def test_persistent_batch_equals_graph_batch(gpu, waves):
    """The whole batch run in one persistent cooperative launch (every tile through the general
    fused sweep, grid barriers between the phases) gives the per-phase graph's bits: waveforms
    and all six final fields of every member, twice in a row."""
    ws = members()[:4]  # the persistent launch takes PEC and CPML members
    print(f"\n[gpu-batch] persistent, {waves}-row tiles", flush=True)
    plans = [solver.Plan(w, kernel="fused", waves=waves) for w in ws]
    batch = solver.Batch(plans)
    ref = [o.cpu().numpy() for o in batch.run()]
    ref_f = [[p.get_field(c).cpu().numpy() for c in range(6)] for p in plans]
    for rep in range(2):
        got = [o.cpu().numpy() for o in batch.run(persistent=True)]
        for m, (a, b) in enumerate(zip(got, ref)):
            assert np.array_equal(a, b), (rep, m)
        for m, p in enumerate(plans):
            for c in range(6):
                assert np.array_equal(p.get_field(c).cpu().numpy(), ref_f[m][c]), (rep, m, c)
    # the captured graph still replays after the persistent runs
    again = [o.cpu().numpy() for o in batch.run()]
    for a, b in zip(again, ref):
        assert np.array_equal(a, b)
    batch.close()
    for p in plans:
        p.close()


def test_persistent_batch_rejects_unsupported_members(gpu):
    ws = members()  # includes a Mur member
    plans = [solver.Plan(w) for w in ws]
    batch = solver.Batch(plans)
    with pytest.raises(_native.ChfError) as e:
        batch.run(persistent=True)
    assert e.value.status == "CHF_EUNSUPPORTED"
    batch.close()
    for p in plans:
        p.close()
