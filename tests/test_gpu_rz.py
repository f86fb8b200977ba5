"""GPU parity of the axisymmetric (r, z) path (include/chfdtd_rz.h) against the FP64 oracle.

FP32 arithmetic against FP64: waveforms and fields within rel. L2 1e-5; every tile shape gives
the same bits; graph replays equal the eager run; at the 8192 x 8192 size the fields after a
few hundred steps equal an oracle run on the part of the lattice the dependency cone reaches
(one cell per step), and are exactly zero outside it.
"""
import math

import numpy as np
import pytest
import torch

from oracle import rz_oracle as R
from paper_1001_5341_amd import _native as N
from paper_1001_5341_amd import solver
from paper_1001_5341_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


_cache = {}


def oracle_run(w):
    key = (w.name, w.nr, w.nz, w.n_steps, w.bc)
    if key not in _cache:
        st = R.RZState(w)
        out = np.zeros((w.n_obs, 2, w.n_steps))
        for n in range(w.n_steps):
            out[:, :, n] = st.step()
        _cache[key] = (out, st.er.copy(), st.ez.copy(), st.hp.copy())
    return _cache[key]


@pytest.fixture(scope="module")
def small_mur():
    return W.rz_small(bc="mur1")


@pytest.fixture(scope="module")
def small_pec():
    return W.rz_small(bc="pec", nr=190, nz=260, n_steps=400, n_obs=6).replace(name="rz-small-pec")


@pytest.mark.parametrize("fixture", ["small_mur", "small_pec"])
def test_waveforms_and_fields_match_oracle(fixture, request):
    w = request.getfixturevalue(fixture)
    print(f"rz parity {w.name} {w.nr}x{w.nz} steps={w.n_steps}", flush=True)
    ref, er, ez, hp = oracle_run(w)
    plan = solver.RZPlan(w)
    try:
        got = plan.run().cpu().numpy()
        assert np.isfinite(got).all()
        assert np.abs(ref).max() > 0
        assert rel_l2(got, ref) <= TOL
        per_obs = [rel_l2(got[o], ref[o]) for o in range(w.n_obs)]
        print("rel L2 per observer", np.array(per_obs), flush=True)
        assert max(per_obs) <= TOL, per_obs
        for comp, want in ((0, er), (1, ez), (2, hp)):
            f = plan.get_field(comp).cpu().numpy()
            assert rel_l2(f, want) <= TOL, comp
    finally:
        plan.close()


# (vx, waves per workgroup, z chunk, Yee steps per launch)
SHAPES = [(1, 1, 1, 1), (1, 2, 2, 1), (1, 2, 7, 1), (2, 8, 5, 1), (4, 4, 32, 1), (4, 4, 32, 2), (4, 1, 600, 2),
          (4, 2, 1, 2), (4, 8, 2, 2), (8, 1, 13, 1), (8, 1, 13, 2), (8, 2, 64, 2)]


@pytest.mark.parametrize("n_steps", [260, 261])
def test_tile_shapes_bitwise_equal(small_mur, n_steps):
    """Every tile shape, with one or two Yee steps per launch (an odd count ends on a one-step
    launch), gives the same waveforms and fields bit for bit."""
    w = small_mur.replace(n_steps=n_steps)
    outs, fields = [], []
    for vx, waves, zc, spl in SHAPES:
        print(f"rz shape vx={vx} waves={waves} z_chunk={zc} steps/launch={spl}", flush=True)
        plan = solver.RZPlan(w, vx=vx, waves=waves, zchunk=zc, steps_per_launch=spl)
        try:
            outs.append(plan.run().cpu())
            fields.append(torch.stack([plan.get_field(c) for c in range(3)]).cpu())
        finally:
            plan.close()
    for o, f in zip(outs[1:], fields[1:]):
        assert torch.equal(o, outs[0])
        assert torch.equal(f, fields[0])


def test_graph_replays_equal_eager(small_mur):
    w = small_mur.replace(n_steps=200)
    plan = solver.RZPlan(w)
    try:
        eager = plan.run()
        out = plan.new_waveforms()
        for rep in range(3):
            out.zero_()
            plan.run(out=out, graph=True)
            torch.cuda.synchronize()
            assert torch.equal(out, eager), rep
            plan.run()  # eager work between replays
    finally:
        plan.close()


def test_profile_override_and_chunked_forward(small_mur):
    """q_bins from the device replaces the plan's profile; a run split into pieces writes the
    same columns as one call."""
    w = small_mur.replace(n_steps=300)
    q2 = w.q_bins * np.linspace(0.5, 1.5, len(w.q_bins))
    ref = oracle_run(w.replace(q_bins=q2, name="rz-q2"))[0]
    plan = solver.RZPlan(w)
    try:
        qd = torch.tensor(q2, dtype=torch.float64, device=plan.device)
        a = plan.run(q_bins=qd)
        assert rel_l2(a.cpu().numpy(), ref) <= TOL
        b = plan.new_waveforms()
        plan.reset()
        for lo, hi in ((0, 1), (1, 120), (120, 300)):
            plan.forward(hi - lo, b, lo, q_bins=qd)
        plan.sync()
        assert torch.equal(a, b)
    finally:
        plan.close()


@pytest.mark.parametrize("nr,nz", [(4, 4), (5, 130), (65, 4), (257, 33), (3001, 41)])
def test_ragged_and_degenerate_sizes(nr, nz):
    """Smallest lattices, one node beyond a wave, rows wider than a workgroup; random fields
    evolved without a source against the oracle."""
    d = 0.01
    w = W.RZWorkload(name=f"rz-edge-{nr}x{nz}", nr=nr, nz=nz, n_steps=25, dr=d, dz=d,
                     dt=W.courant_dt(d, d, d), bc="mur1", src_on=False, q_bins=np.zeros(2),
                     obs_rz=np.zeros((0, 2)))
    rng = np.random.default_rng(nr * 7 + nz)
    st = R.RZState(w)
    st.er[1:-1, :-1] = rng.standard_normal((nz - 2, nr - 1))
    st.ez[:-1, :-1] = rng.standard_normal((nz - 1, nr - 1))
    st.hp[:-1, :-1] = rng.standard_normal((nz - 1, nr - 1)) / 377.0
    init = (st.er.copy(), st.ez.copy(), st.hp.copy())
    for _ in range(w.n_steps):
        st.step()
    plan = solver.RZPlan(w)
    try:
        for c in range(3):
            plan.set_field(c, torch.tensor(init[c], dtype=torch.float32))
        plan.forward(w.n_steps)
        plan.sync()
        for c, want in enumerate((st.er, st.ez, st.hp)):
            assert rel_l2(plan.get_field(c).cpu().numpy(), want) <= TOL, c
    finally:
        plan.close()


def test_watchdog_reports_nan(small_mur):
    w = small_mur.replace(n_steps=20)
    plan = solver.RZPlan(w, nan_watch=True)
    try:
        f = torch.zeros((w.nz, w.nr))
        r, z = w.obs_rz[0]
        k, i = int(z / w.dz), int(r / w.dr)
        f[k - 3:k + 3, i - 3:i + 3] = float("nan")  # around the first observer's stencil
        plan.set_field(1, f)
        plan.forward(w.n_steps, plan.new_waveforms())
        with pytest.raises(N.ChfError) as e:
            plan.sync()
        assert e.value.status == "CHF_ENAN"
        plan.run()  # reset clears the flag
    finally:
        plan.close()


def test_fullsize_8192_dependency_cone():
    """rz-8192 (the paper's largest grid) in the default launch shape: after T steps the
    fields equal an oracle run on the part of the lattice that the source's dependency cone
    reaches, and are exactly zero everywhere else."""
    w = W.rz_paper_grid(8192)
    T = 500
    print(f"rz full size {w.nr}x{w.nz}, {T} steps", flush=True)
    plan = solver.RZPlan(w.replace(n_steps=T))
    try:
        plan.run()
        n_src = plan.info()["n_src"]
        fields = [plan.get_field(c) for c in range(3)]
    finally:
        plan.close()
    z0 = int(math.ceil(w.z_entry / w.dz))
    nr_c = n_src + T + 8
    nz_c = z0 + int(math.ceil(T * W.C0 * w.dt / w.dz)) + int(math.ceil(w.cut_sigmas * w.sigma_z / w.dz)) + T + 8
    crop = w.replace(nr=nr_c, nz=nz_c, n_steps=T, obs_rz=np.zeros((0, 2)), name="rz-8192-cone")
    st = R.RZState(crop)
    for _ in range(T):
        st.update_h()
        st.update_e()
    for c, want in enumerate((st.er, st.ez, st.hp)):
        f = fields[c]
        inner = f[:nz_c - 1, :nr_c - 1].cpu().numpy()
        assert rel_l2(inner, want[:-1, :-1]) <= TOL, c
        # the crop's own walls were never reached: its outermost rows and columns are zero
        assert not np.any(want[-2:, :]) and not np.any(want[:, -2:])
        outside = f.clone()
        outside[:nz_c - 1, :nr_c - 1] = 0
        assert int(torch.count_nonzero(outside)) == 0, c


@pytest.mark.parametrize("nr,vx,sigma_r", [(65, 1, 0.02), (129, 2, 0.02), (257, 4, 0.05), (14, 4, 0.04)])
def test_wall_at_wave_start_and_source_at_wall(nr, vx, sigma_r):
    """The r wall as the first node of a wave (its Mur value then comes from a kernel of its
    own), and a source patch reaching the node next to the wall, against the oracle."""
    d = 0.01
    nz = 160
    zb = np.arange(0.0, 2.0, d)
    q = -1e-10 * np.exp(-0.5 * ((zb - 0.5) / 0.1) ** 2)
    rr = min(0.5 * (nr - 1) * d, 0.3)
    obs = np.array([[rr, 0.6], [0.5 * rr, 0.9], [0.8 * rr, 1.2]])
    w = W.RZWorkload(name=f"rz-wall-{nr}-{vx}", nr=nr, nz=nz, n_steps=220, dr=d, dz=d,
                     dt=W.courant_dt(d, d, d), bc="mur1", z_entry=0.05, sigma_r=sigma_r, sigma_z=0.01,
                     z_bin0=0.0, dz_bin=d, q_bins=q, obs_rz=obs)
    ref, er, ez, hp = oracle_run(w)
    plan = solver.RZPlan(w, vx=vx, waves=2, zchunk=9)
    try:
        got = plan.run().cpu().numpy()
        assert rel_l2(got, ref) <= TOL
        for comp, want in ((0, er), (1, ez), (2, hp)):
            assert rel_l2(plan.get_field(comp).cpu().numpy(), want) <= TOL, comp
    finally:
        plan.close()


@pytest.mark.parametrize("storage,tol", [("fp16", 1e-2), ("bf16", 1e-1)])
def test_16bit_storage_against_oracle(small_mur, storage, tol):
    """FP32 arithmetic on FP16 / BF16 fields (fixed power-of-two scales), against the FP64 oracle.
    FP16 is held to the 1e-2 storage gate.  BF16 (8-bit mantissa) does not meet that gate on this
    path: its bound here is an error-envelope regression check at about five times the measured
    1.9e-2, not a parity claim."""
    w = small_mur
    ref = oracle_run(w)[0]
    plan = solver.RZPlan(w, storage=storage)
    try:
        got = plan.run().cpu().numpy()
        info = plan.info()
    finally:
        plan.close()
    err = rel_l2(got, ref)
    print(f"{storage}: rel L2 {err:.3e}, scales {info['scale_e']} {info['scale_h']}", flush=True)
    assert np.isfinite(got).all() and err <= tol


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_16bit_one_and_two_steps_per_launch_bitwise(small_mur, storage):
    """With fixed scales the two-step kernel rounds its intermediate level exactly as a store and
    load would, so one and two steps per launch give the same bits."""
    w = small_mur.replace(n_steps=301)
    outs = []
    for spl, waves, zc in ((1, 4, 32), (2, 2, 9)):
        plan = solver.RZPlan(w, storage=storage, steps_per_launch=spl, waves=waves, zchunk=zc)
        try:
            outs.append((plan.run().cpu(), torch.stack([plan.get_field(c) for c in range(3)]).cpu()))
        finally:
            plan.close()
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])


def test_fp16_dynamic_scaling(small_mur):
    """Per-launch scales chosen from the previous level's maxima: within the FP16 tolerance of the
    oracle from the automatic start, and still there when the fixed scale would be far too small
    (a 2^-32 fixed scale flushes the fields to zero in FP16)."""
    w = small_mur
    ref = oracle_run(w)[0]
    res = {}
    for name, kw in (("dynamic", dict(dynamic_scaling=True)), ("dynamic-2", dict(dynamic_scaling=True, steps_per_launch=1)),
                     ("static-tiny", dict(scale_e=2.0 ** -32, scale_h=2.0 ** -24))):
        plan = solver.RZPlan(w, storage="fp16", **kw)
        try:
            got = plan.run().cpu().numpy()
        finally:
            plan.close()
        res[name] = rel_l2(got, ref) if np.isfinite(got).all() else float("inf")
    print(res, flush=True)
    assert res["dynamic"] <= 2e-2 and res["dynamic-2"] <= 2e-2
    assert res["static-tiny"] > 0.5
