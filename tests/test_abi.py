"""C-ABI checks that need no GPU: the library loads, exports every declared entry point, and
chf_plan_create validates descriptors on the host."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_1001_5341_amd import _native as N
from paper_1001_5341_amd import solver
from paper_1001_5341_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    inc = os.path.join(ROOT, "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chf_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = N.lib()
    names = declared_symbols()
    assert "chf_plan_create" in names and "chf_forward" in names and "chf_rz_forward" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(N.EXPORTED)
    assert L.chf_abi_version() == 3


def _status(w, **kw):
    try:
        h = solver.create_plan_handle(w, **kw)
    except N.ChfError as e:
        return e.status
    N.lib().chf_plan_destroy(h)
    return "CHF_OK"


def test_valid_plans_accepted():
    assert _status(W.gaussian_cube(1)) == "CHF_OK"
    assert _status(W.small_shower()) == "CHF_OK"
    assert _status(W.small_shower(), storage="bf16") == "CHF_OK"
    assert _status(W.small_shower(), storage="bf16x") == "CHF_OK"
    assert _status(W.small_shower(), kernel="split") == "CHF_OK"


def test_cfl_violation_rejected():
    w = W.gaussian_cube(1)
    dt_lim = 1.0 / (W.C0 / W.N_ICE * np.sqrt(3) / w.dx)
    assert _status(w.replace(dt=dt_lim * 0.999)) == "CHF_OK"
    assert _status(w.replace(dt=dt_lim * 1.001)) == "CHF_ECFL"


def test_observer_outside_interior_rejected():
    w = W.small_shower()
    obs = w.obs_xyz.copy()
    obs[0, 0] = (w.npml - 0.5) * w.dx  # stencil in the CPML
    assert _status(w.replace(obs_xyz=obs)) == "CHF_EDOMAIN"
    obs[0, 0] = -1.0
    assert _status(w.replace(obs_xyz=obs)) == "CHF_EDOMAIN"


def test_source_outside_grid_rejected():
    w = W.small_shower()
    assert _status(w.replace(x_axis=-1.0)) == "CHF_EDOMAIN"


def test_bad_descriptors_rejected():
    w = W.small_shower()
    assert _status(w.replace(nx=2)) == "CHF_EINVAL"
    assert _status(w.replace(dx=0.0)) == "CHF_EINVAL"
    assert _status(w.replace(npml=40)) == "CHF_EINVAL"
    assert _status(w.replace(eps_r=-1.0)) == "CHF_EINVAL"
    assert _status(w, rows=3) == "CHF_EINVAL"
    assert _status(w.replace(sigma_r=0.0)) == "CHF_EINVAL"


def test_fused_sweep_width_limit():
    w = W.gaussian_cube(1, n=24, n_steps=2)
    big = w.replace(nx=600, x_axis=0.5 * 599 * w.dx, obs_xyz=w.obs_xyz + [0.5 * (599 - 23) * w.dx, 0, 0])
    assert _status(big, kernel="fused") == "CHF_EUNSUPPORTED"
    assert _status(big, kernel="split") == "CHF_OK"
    assert _status(big) == "CHF_OK"  # auto picks the split sweeps


def test_prefetching_sweep_limits():
    """The prefetching sweep holds more registers per wave (3 waves per SIMD): at most 12 waves
    per workgroup and 4 nodes per lane; the plan reports it as its kernel."""
    w = W.small_shower()
    for waves in (4, 7, 8, 11):
        assert _status(w, kernel="fused_prefetch", waves=waves) == "CHF_OK"
    assert _status(w, kernel="fused", waves=11) == "CHF_OK"
    assert _status(w, kernel="fused_prefetch", waves=15) == "CHF_EINVAL"
    for waves in (5, 9, 12, 16):
        assert _status(w, kernel="fused", waves=waves) == "CHF_EINVAL"
    wide = w.replace(nx=300, x_axis=0.5 * 299 * w.dx, obs_xyz=w.obs_xyz + [0.5 * (299 - w.nx + 1) * w.dx, 0, 0])
    assert _status(wide, kernel="fused", waves=7) == "CHF_OK"
    assert _status(wide, kernel="fused", waves=11) == "CHF_EINVAL"
    assert _status(wide, kernel="fused_prefetch", waves=7) == "CHF_EINVAL"
    h = solver.create_plan_handle(w, kernel="fused_prefetch", waves=8, zchunk=16)
    try:
        info = N.PlanInfo()
        assert N.lib().chf_plan_get_info(h, ct.byref(info)) == 0
        assert (info.kernel, info.waves_per_block, info.z_chunk) == (3, 8, 16)
    finally:
        N.lib().chf_plan_destroy(h)


def test_null_pointers_rejected():
    L = N.lib()
    h = ct.c_void_p()
    assert L.chf_plan_create(None, None, None, None, None, None, ct.byref(h)) == -1
    assert L.chf_plan_workspace_bytes(None, None) == -1
    assert L.chf_forward(None, None, None, None, 1, 0, 1) == -1


def test_workspace_size_and_binding_checks():
    L = N.lib()
    h = solver.create_plan_handle(W.small_shower())
    try:
        n = ct.c_uint64()
        assert L.chf_plan_workspace_bytes(h, ct.byref(n)) == 0
        info = N.PlanInfo()
        assert L.chf_plan_get_info(h, ct.byref(info)) == 0
        assert n.value == info.workspace_bytes > info.field_bytes > 0
        # too small, then misaligned: both refused before any device call
        assert L.chf_plan_bind_workspace(h, ct.c_void_p(4096), n.value - 1, None) == -4
        assert L.chf_plan_bind_workspace(h, ct.c_void_p(4096 + 8), n.value, None) == -1
        # use before binding
        assert L.chf_forward(h, None, None, None, 1, 0, 1) == -8
    finally:
        L.chf_plan_destroy(h)


def test_plan_info_layout():
    h = solver.create_plan_handle(W.single_shower())
    try:
        info = N.PlanInfo()
        assert N.lib().chf_plan_get_info(h, ct.byref(info)) == 0
        assert info.kernel == 2 and info.vx == 4 and info.pitch == 256
        # 48 B of fields + the CPML psi share of 256x256x2048 with 10-cell layers
        assert abs(info.bytes_per_cell_update - (48 + 32 * (20 / 256 + 20 / 256 + 20 / 2048))) < 1e-9
        assert info.scale_h == 256.0 and info.scale_e == 1.0
    finally:
        N.lib().chf_plan_destroy(h)


def test_snapshot_size_and_adjoint_state_checks():
    """Host-side checks of the checkpoint entry points (no device call is made)."""
    h = solver.create_plan_handle(W.small_shower())
    try:
        info = N.PlanInfo()
        assert N.lib().chf_plan_get_info(h, ct.byref(info)) == 0
        n = ct.c_uint64()
        assert N.lib().chf_plan_state_bytes(h, ct.byref(n)) == 0
        # a snapshot is both field levels, every psi array and the dynamic-scaling words
        assert n.value == info.field_bytes + info.psi_bytes + 256
        step = ct.c_int32()
        assert N.STATUS[N.lib().chf_plan_save_state(h, None, ct.c_void_p(1), ct.byref(step))] == "CHF_ESTATE"
        assert N.STATUS[N.lib().chf_adjoint_steps(h, None, ct.c_void_p(1), ct.c_void_p(1), 0, 5)] == "CHF_ESTATE"
        assert N.STATUS[N.lib().chf_plan_load_state(h, None, None, 0)] == "CHF_EINVAL"
        one = ct.c_void_p(1)
        assert N.STATUS[N.lib().chf_adjoint_steps_eps(h, None, one, one, 0, 5, None, one)] == "CHF_EINVAL"
        assert N.STATUS[N.lib().chf_adjoint_steps_eps(h, None, one, one, 0, 5, one, None)] == "CHF_EINVAL"
        assert N.STATUS[N.lib().chf_adjoint_steps_eps(h, None, one, one, 0, 5, one, one)] == "CHF_ESTATE"
        L = N.lib()
        h2 = solver.create_plan_handle(W.small_shower())
        try:
            def ck(a, b, snaps=one, every=4, lv=None, dg=None):
                return N.STATUS[L.chf_adjoint_checkpointed(a, b, None, None, one, one, every, snaps, 1 << 40, lv, dg)]
            assert ck(h, None) == "CHF_EINVAL"
            assert ck(h, h) == "CHF_EINVAL"            # the recomputation needs a second plan
            assert ck(h, h2, snaps=None) == "CHF_EINVAL"
            assert ck(h, h2, lv=one) == "CHF_EINVAL"    # levels without the permittivity output
            assert ck(h, h2) == "CHF_ESTATE"            # no workspace bound
        finally:
            L.chf_plan_destroy(h2)
    finally:
        N.lib().chf_plan_destroy(h)


def _rz_status(w, **kw):
    try:
        h = solver.create_rz_plan_handle(w, **kw)
    except N.ChfError as e:
        return e.status
    N.lib().chf_rz_plan_destroy(h)
    return "CHF_OK"


def test_dynamic_scaling_validation():
    """Per-launch scaling is accepted for FP16 storage with the fused one- and two-step sweeps
    (PEC or CPML walls) and rejected elsewhere, on the host."""
    w = W.small_shower()
    for kernel in ("auto", "fused", "fused_prefetch", "fused2"):
        assert _status(w, storage="fp16", kernel=kernel, dynamic_scaling=True) == "CHF_OK", kernel
    assert _status(w.replace(nx=300), storage="fp16", kernel="fused_prefetch", dynamic_scaling=True) == "CHF_OK"
    assert _status(w.replace(bc="pec", npml=0), storage="fp16", dynamic_scaling=True) == "CHF_OK"
    assert _status(w, storage="fp32", dynamic_scaling=True) == "CHF_EUNSUPPORTED"
    assert _status(w, storage="bf16", dynamic_scaling=True) == "CHF_EUNSUPPORTED"
    assert _status(w, storage="bf16x", dynamic_scaling=True) == "CHF_EUNSUPPORTED"
    assert _status(w, storage="fp16", kernel="split", dynamic_scaling=True) == "CHF_EUNSUPPORTED"
    assert _status(w, storage="fp16", waves=15, dynamic_scaling=True) == "CHF_EUNSUPPORTED"
    assert _status(W.gaussian_cube(1), storage="fp16", dynamic_scaling=True) == "CHF_EUNSUPPORTED"  # Mur
    h = solver.create_plan_handle(w, storage="fp16", dynamic_scaling=True)
    pi = N.PlanInfo()
    N.check(N.lib().chf_plan_get_info(h, ct.byref(pi)), "info")
    N.lib().chf_plan_destroy(h)
    assert pi.dynamic_scaling == 1


def test_rz_plan_validation():
    w = W.rz_small()
    assert _rz_status(w) == "CHF_OK"
    assert _rz_status(W.rz_paper_grid(8192)) == "CHF_OK"
    assert _rz_status(w.replace(bc="cpml")) == "CHF_EUNSUPPORTED"
    assert _rz_status(w, vx=3) == "CHF_EINVAL"
    assert _rz_status(w, waves=16) == "CHF_EINVAL"
    assert _rz_status(w.replace(nr=3)) == "CHF_EINVAL"
    # stability limit of the (r, z) lattice: the axis raises the radial eigenvalue to 4.85/dr^2
    v = W.C0 / W.N_ICE
    lim = 2.0 / (v * np.sqrt(4.85 / w.dr ** 2 + 4.0 / w.dz ** 2))
    assert _rz_status(w.replace(dt=lim * 0.999)) == "CHF_OK"
    assert _rz_status(w.replace(dt=lim * 1.001)) == "CHF_ECFL"
    for r, z in ((0.3 * w.dr, 1.0), (1.0, (w.nz - 1.2) * w.dz), ((w.nr - 1.2) * w.dr, 1.0)):
        obs = w.obs_rz.copy()
        obs[0] = (r, z)
        assert _rz_status(w.replace(obs_rz=obs)) == "CHF_EDOMAIN"


def test_rz_radial_stability_constant():
    """The largest eigenvalue of the radial operator (E_z -> H_phi -> E_z with the axis disc)
    stays below the 4.85/dr^2 the plan's stability check assumes, for any nr."""
    for nr in (4, 9, 64, 700):
        i = np.arange(nr - 1)
        a = np.where(i == 0, 1.0 / 8.0, i.astype(float))
        D = np.eye(nr - 1, k=1) - np.eye(nr - 1)
        C = np.diag((i + 0.5) / a) - np.diag(((i - 0.5) / a)[1:], k=-1)
        lam = np.max(np.linalg.eigvals(-C @ D).real)
        assert 4.0 < lam < 4.85


def test_rz_storage_and_scaling_validation():
    w = W.rz_small()
    assert _rz_status(w, storage="bf16") == "CHF_OK"
    assert _rz_status(w, storage="fp16", dynamic_scaling=True) == "CHF_OK"
    assert _rz_status(w, storage="bf16", dynamic_scaling=True) == "CHF_EINVAL"
    assert _rz_status(w, dynamic_scaling=True) == "CHF_EINVAL"           # FP32 needs no scales
    assert _rz_status(w, storage="fp16", scale_e=-1.0) == "CHF_EINVAL"
    assert _rz_status(w, vx=2, steps_per_launch=2) == "CHF_EINVAL"       # two steps need vx >= 4
    assert _rz_status(w, vx=2, steps_per_launch=1) == "CHF_OK"


def test_rz_plan_info_reports_storage_and_scales():
    """Automatic scales: BF16 keeps E unscaled and H at the power of two nearest the wave
    impedance of ice (about 212 ohm -> 256); FP16 scales E by a power of two as well."""
    import ctypes as ct

    w = W.rz_small()
    for storage, exp_bytes in (("fp32", 24.0), ("bf16", 12.0), ("fp16", 12.0)):
        h = solver.create_rz_plan_handle(w, storage=storage)
        try:
            info = N.RZInfo()
            N.check(N.lib().chf_rz_get_info(h, ct.byref(info)), "info")
        finally:
            N.lib().chf_rz_plan_destroy(h)
        assert info.bytes_per_cell_update == exp_bytes
        if storage == "bf16":
            assert info.scale_e == 1.0 and info.scale_h == 256.0
        if storage == "fp16":
            assert np.log2(info.scale_e) == int(np.log2(info.scale_e)) and info.scale_h == 256.0 * info.scale_e


def test_bf16x_plan_layout():
    """3 bytes per stored value: the field region is 12 arrays of 3-byte elements, the interior
    sweep's algorithmic bytes 36 per node plus the x-layer psi; FP32's range, so unit scales as
    BF16 has."""
    h = solver.create_plan_handle(W.single_shower(), storage="bf16x")
    try:
        info = N.PlanInfo()
        assert N.lib().chf_plan_get_info(h, ct.byref(info)) == 0
        assert info.storage == 3 and info.pitch == 256
        assert info.field_bytes == 12 * 256 * 256 * 2048 * 3
        assert abs(info.fused_bytes_per_cell - (36 + 32 * 20 / 256)) < 1e-9
        assert info.scale_e == 1.0
    finally:
        N.lib().chf_plan_destroy(h)
    assert _rz_status(W.rz_small(), storage="bf16x") == "CHF_EINVAL"  # the (r, z) scheme does not take it


def _fused_cells(w, **kw):
    h = solver.create_plan_handle(w, **kw)
    try:
        info = N.PlanInfo()
        assert N.lib().chf_plan_get_info(h, ct.byref(info)) == 0
        return info.fused_cells, info.kernel
    finally:
        N.lib().chf_plan_destroy(h)


@pytest.mark.parametrize("bc,npml", [("cpml", 10), ("cpml", 6), ("pec", 0)])
def test_interior_rectangle_starts_at_the_first_clear_row_and_plane(bc, npml):
    """The tile grids are shifted so that the interior rectangle holds every whole tile and
    chunk that fits in the region clear of walls and layers: for the one-step sweep the tile's
    rows and the row below it, for the two-step pass the computed rows and staged planes (two
    below, one above)."""
    for ny, nz in ((44, 72), (60, 150), (57, 131)):
        w = W.small_shower(seed=3, nx=64, ny=ny, nz=nz, n_steps=10, n_obs=2, npml=max(npml, 6), bc=bc)
        nl = w.npml if bc == "cpml" else 0
        fy0, fy1, fz0, fz1 = max(1, nl), ny - 2 - nl, max(1, nl), nz - 2 - nl
        for waves, zc in ((4, 7), (7, 8), (8, 12), (11, 5), (5, 9)):
            if waves == 5:
                continue  # 5 rows is the split-row tile of 257-512-node rows
            ty, tz = (fy1 - fy0) // waves, (fz1 - fz0 + 1) // zc
            cells, kern = _fused_cells(w, kernel="fused", waves=waves, zchunk=zc)
            assert cells == (ty * waves * tz * zc * w.nx if ty > 0 and tz > 0 else 0), (ny, nz, waves, zc)
            if waves in (4, 7, 8):
                ty, tz = (fy1 - fy0 - 2) // waves, (fz1 - fz0 - 2) // zc
                cells, kern = _fused_cells(w, kernel="fused2", waves=waves, zchunk=zc)
                assert kern == 4
                assert cells == (ty * waves * tz * zc * w.nx if ty > 0 and tz > 0 else 0), (ny, nz, waves, zc)
