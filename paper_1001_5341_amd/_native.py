"""ctypes declarations of the C ABI in include/chfdtd.h and include/chfdtd_rz.h (argument
marshalling only).

Loading fails loudly when libchfdtd.so is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchfdtd.so")

CHF_OK = 0
STATUS = {0: "CHF_OK", -1: "CHF_EINVAL", -2: "CHF_ECFL", -3: "CHF_EDOMAIN", -4: "CHF_ENOMEM",
          -5: "CHF_EHIP", -6: "CHF_ENAN", -7: "CHF_EUNSUPPORTED", -8: "CHF_ESTATE"}
STORAGE = {"fp32": 0, "bf16": 1, "fp16": 2, "bf16x": 3}
BC = {"pec": 0, "mur1": 1, "cpml": 2}
KERNEL = {"auto": 0, "split": 1, "fused": 2, "fused_prefetch": 3, "fused2": 4}

EXPORTED = [
    "chf_plan_create", "chf_plan_destroy", "chf_plan_workspace_bytes", "chf_plan_bind_workspace",
    "chf_plan_reset", "chf_forward", "chf_forward_timed", "chf_forward_graph", "chf_adjoint",
    "chf_adjoint_begin", "chf_adjoint_steps", "chf_adjoint_steps_eps", "chf_adjoint_checkpointed", "chf_adjoint_source_params", "chf_plan_state_bytes",
    "chf_plan_save_state",
    "chf_plan_load_state", "chf_plan_sync",
    "chf_plan_get_field", "chf_plan_set_field", "chf_plan_get_info", "chf_batch_create",
    "chf_batch_workspace_bytes", "chf_batch_bind_workspace", "chf_batch_run", "chf_batch_run_persistent",
    "chf_batch_destroy",
    "chf_status_str", "chf_last_error", "chf_abi_version", "chf_forward_scratch", "chf_scratch_bytes",
    "chf_stream_copy",
    "chf_rz_plan_create", "chf_rz_plan_destroy", "chf_rz_workspace_bytes", "chf_rz_bind_workspace",
    "chf_rz_reset", "chf_rz_forward", "chf_rz_forward_timed", "chf_rz_forward_graph", "chf_rz_sync",
    "chf_rz_get_field", "chf_rz_set_field", "chf_rz_get_info",
    "chf_spectrum", "chf_spectrum_project", "chf_geometry_rz", "chf_geometry_xyz", "chf_far_field_1d",
]


class Grid(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32), ("n_steps", ct.c_int32),
                ("dx", ct.c_double), ("dy", ct.c_double), ("dz", ct.c_double), ("dt", ct.c_double)]


class Medium(ct.Structure):
    _fields_ = [("eps_r", ct.c_double), ("mu_r", ct.c_double), ("sigma", ct.c_double)]


class Boundary(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("npml", ct.c_int32), ("poly_m", ct.c_double),
                ("sigma_scale", ct.c_double), ("kappa_max", ct.c_double), ("alpha_max", ct.c_double)]


class Source(ct.Structure):
    _fields_ = [("x_axis", ct.c_double), ("y_axis", ct.c_double), ("z_entry", ct.c_double),
                ("t_entry", ct.c_double), ("beta", ct.c_double), ("sigma_r", ct.c_double),
                ("sigma_z", ct.c_double), ("cut_sigmas", ct.c_double), ("n_bins", ct.c_int32),
                ("pad0", ct.c_int32), ("z_bin0", ct.c_double), ("dz_bin", ct.c_double),
                ("q_bins", ct.POINTER(ct.c_double))]


class Observers(ct.Structure):
    _fields_ = [("n_obs", ct.c_int32), ("pad0", ct.c_int32), ("xyz", ct.POINTER(ct.c_double))]


class Exec(ct.Structure):
    _fields_ = [("storage", ct.c_int32), ("kernel", ct.c_int32), ("rows_per_wave", ct.c_int32),
                ("waves_per_block", ct.c_int32), ("z_chunk", ct.c_int32), ("nan_watch", ct.c_int32),
                ("scale_e", ct.c_double), ("scale_h", ct.c_double), ("dynamic_scaling", ct.c_int32),
                ("pad0", ct.c_int32)]


class PlanInfo(ct.Structure):
    _fields_ = [("kernel", ct.c_int32), ("storage", ct.c_int32), ("vx", ct.c_int32),
                ("rows_per_wave", ct.c_int32), ("waves_per_block", ct.c_int32),
                ("z_chunk", ct.c_int32), ("pitch", ct.c_int32), ("n_blocks", ct.c_int32),
                ("scale_e", ct.c_double), ("scale_h", ct.c_double), ("field_bytes", ct.c_uint64),
                ("psi_bytes", ct.c_uint64), ("workspace_bytes", ct.c_uint64),
                ("bytes_per_cell_update", ct.c_double), ("fused_cells", ct.c_uint64),
                ("fused_bytes_per_cell", ct.c_double), ("steps_per_launch", ct.c_int32),
                ("waves_per_row", ct.c_int32), ("pass_bytes_per_cell", ct.c_double),
                ("dynamic_scaling", ct.c_int32), ("pad0", ct.c_int32)]


class RZGrid(ct.Structure):
    _fields_ = [("nr", ct.c_int32), ("nz", ct.c_int32), ("n_steps", ct.c_int32), ("pad0", ct.c_int32),
                ("dr", ct.c_double), ("dz", ct.c_double), ("dt", ct.c_double)]


class RZSource(ct.Structure):
    _fields_ = [("z_entry", ct.c_double), ("t_entry", ct.c_double), ("beta", ct.c_double),
                ("sigma_r", ct.c_double), ("sigma_z", ct.c_double), ("cut_sigmas", ct.c_double),
                ("n_bins", ct.c_int32), ("pad0", ct.c_int32), ("z_bin0", ct.c_double),
                ("dz_bin", ct.c_double), ("q_bins", ct.POINTER(ct.c_double))]


class RZObservers(ct.Structure):
    _fields_ = [("n_obs", ct.c_int32), ("pad0", ct.c_int32), ("rz", ct.POINTER(ct.c_double))]


class RZExec(ct.Structure):
    _fields_ = [("bc", ct.c_int32), ("vx", ct.c_int32), ("waves_per_block", ct.c_int32),
                ("z_chunk", ct.c_int32), ("nan_watch", ct.c_int32), ("steps_per_launch", ct.c_int32),
                ("storage", ct.c_int32), ("dynamic_scaling", ct.c_int32), ("scale_e", ct.c_double),
                ("scale_h", ct.c_double)]


class RZInfo(ct.Structure):
    _fields_ = [("vx", ct.c_int32), ("waves_per_block", ct.c_int32), ("z_chunk", ct.c_int32),
                ("pitch", ct.c_int32), ("n_blocks", ct.c_int32), ("n_src", ct.c_int32),
                ("steps_per_launch", ct.c_int32), ("storage", ct.c_int32),
                ("dynamic_scaling", ct.c_int32), ("pad0", ct.c_int32),
                ("field_bytes", ct.c_uint64), ("workspace_bytes", ct.c_uint64),
                ("bytes_per_cell_update", ct.c_double), ("scale_e", ct.c_double), ("scale_h", ct.c_double)]


class FarFieldParams(ct.Structure):
    _fields_ = [("n_index", ct.c_double), ("beta", ct.c_double), ("z_entry", ct.c_double),
                ("t_entry", ct.c_double), ("z_origin", ct.c_double)]


class ChfError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS.get(code, code)} ({detail})")
        self.code = code
        self.status = STATUS.get(code, str(code))


_lock = threading.Lock()
_lib = None


def lib():
    """The loaded libchfdtd.so.  Raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1001_5341_amd/build.py "
                               "(there is no non-HIP fallback)")
        L = ct.CDLL(LIB_PATH)
        vp, dp = ct.c_void_p, ct.POINTER(ct.c_double)
        L.chf_plan_create.restype = ct.c_int
        L.chf_plan_create.argtypes = [ct.POINTER(Grid), ct.POINTER(Medium), ct.POINTER(Boundary),
                                      ct.POINTER(Source), ct.POINTER(Observers), ct.POINTER(Exec),
                                      ct.POINTER(vp)]
        L.chf_plan_destroy.restype = None
        L.chf_plan_destroy.argtypes = [vp]
        L.chf_plan_workspace_bytes.restype = ct.c_int
        L.chf_plan_workspace_bytes.argtypes = [vp, ct.POINTER(ct.c_uint64)]
        L.chf_plan_bind_workspace.restype = ct.c_int
        L.chf_plan_bind_workspace.argtypes = [vp, vp, ct.c_uint64, vp]
        L.chf_plan_reset.restype = ct.c_int
        L.chf_plan_reset.argtypes = [vp, vp]
        L.chf_forward.restype = ct.c_int
        L.chf_forward.argtypes = [vp, vp, vp, vp, ct.c_int32, ct.c_int32, ct.c_int32]
        L.chf_forward_timed.restype = ct.c_int
        L.chf_forward_timed.argtypes = [vp, vp, vp, vp, ct.c_int32, ct.c_int32, ct.c_int32,
                                        ct.POINTER(ct.c_double)]
        L.chf_forward_graph.restype = ct.c_int
        L.chf_forward_graph.argtypes = [vp, vp, vp, vp]
        L.chf_forward_scratch.restype = ct.c_int
        L.chf_forward_scratch.argtypes = [vp, vp, vp, vp]
        L.chf_scratch_bytes.restype = ct.c_uint64
        L.chf_scratch_bytes.argtypes = []
        L.chf_stream_copy.restype = ct.c_int
        L.chf_stream_copy.argtypes = [vp, vp, ct.c_uint64, ct.c_int32, ct.c_int32, vp]
        L.chf_adjoint.restype = ct.c_int
        L.chf_adjoint.argtypes = [vp, vp, vp, vp]
        L.chf_adjoint_begin.restype = ct.c_int
        L.chf_adjoint_begin.argtypes = [vp, vp, vp]
        L.chf_adjoint_steps.restype = ct.c_int
        L.chf_adjoint_steps.argtypes = [vp, vp, vp, vp, ct.c_int32, ct.c_int32]
        L.chf_adjoint_steps_eps.restype = ct.c_int
        L.chf_adjoint_steps_eps.argtypes = [vp, vp, vp, vp, ct.c_int32, ct.c_int32, vp, vp]
        L.chf_adjoint_checkpointed.restype = ct.c_int
        L.chf_adjoint_checkpointed.argtypes = [vp, vp, vp, vp, vp, vp, ct.c_int32, vp, ct.c_uint64, vp, vp]
        L.chf_adjoint_source_params.restype = ct.c_int
        L.chf_adjoint_source_params.argtypes = [vp, vp, vp, vp, vp, vp]
        L.chf_plan_state_bytes.restype = ct.c_int
        L.chf_plan_state_bytes.argtypes = [vp, ct.POINTER(ct.c_uint64)]
        L.chf_plan_save_state.restype = ct.c_int
        L.chf_plan_save_state.argtypes = [vp, vp, vp, ct.POINTER(ct.c_int32)]
        L.chf_plan_load_state.restype = ct.c_int
        L.chf_plan_load_state.argtypes = [vp, vp, vp, ct.c_int32]
        L.chf_plan_sync.restype = ct.c_int
        L.chf_plan_sync.argtypes = [vp, vp]
        L.chf_plan_get_field.restype = ct.c_int
        L.chf_plan_get_field.argtypes = [vp, vp, ct.c_int32, vp]
        L.chf_plan_set_field.restype = ct.c_int
        L.chf_plan_set_field.argtypes = [vp, vp, ct.c_int32, vp]
        L.chf_plan_get_info.restype = ct.c_int
        L.chf_plan_get_info.argtypes = [vp, ct.POINTER(PlanInfo)]
        L.chf_batch_create.restype = ct.c_int
        L.chf_batch_create.argtypes = [ct.c_int32, ct.POINTER(vp), ct.POINTER(vp)]
        L.chf_batch_workspace_bytes.restype = ct.c_int
        L.chf_batch_workspace_bytes.argtypes = [vp, ct.POINTER(ct.c_uint64)]
        L.chf_batch_bind_workspace.restype = ct.c_int
        L.chf_batch_bind_workspace.argtypes = [vp, vp, ct.c_uint64, vp]
        L.chf_batch_run.restype = ct.c_int
        L.chf_batch_run.argtypes = [vp, vp, ct.POINTER(vp)]
        L.chf_batch_run_persistent.restype = ct.c_int
        L.chf_batch_run_persistent.argtypes = [vp, vp, ct.POINTER(vp)]
        L.chf_batch_destroy.restype = None
        L.chf_batch_destroy.argtypes = [vp]
        L.chf_status_str.restype = ct.c_char_p
        L.chf_status_str.argtypes = [ct.c_int]
        L.chf_last_error.restype = ct.c_char_p
        L.chf_last_error.argtypes = []
        L.chf_abi_version.restype = ct.c_int32
        L.chf_abi_version.argtypes = []
        L.chf_rz_plan_create.restype = ct.c_int
        L.chf_rz_plan_create.argtypes = [ct.POINTER(RZGrid), ct.POINTER(Medium), ct.POINTER(RZSource),
                                         ct.POINTER(RZObservers), ct.POINTER(RZExec), ct.POINTER(vp)]
        L.chf_rz_plan_destroy.restype = None
        L.chf_rz_plan_destroy.argtypes = [vp]
        L.chf_rz_workspace_bytes.restype = ct.c_int
        L.chf_rz_workspace_bytes.argtypes = [vp, ct.POINTER(ct.c_uint64)]
        L.chf_rz_bind_workspace.restype = ct.c_int
        L.chf_rz_bind_workspace.argtypes = [vp, vp, ct.c_uint64, vp]
        L.chf_rz_reset.restype = ct.c_int
        L.chf_rz_reset.argtypes = [vp, vp]
        L.chf_rz_forward.restype = ct.c_int
        L.chf_rz_forward.argtypes = [vp, vp, vp, vp, ct.c_int32, ct.c_int32, ct.c_int32]
        L.chf_rz_forward_timed.restype = ct.c_int
        L.chf_rz_forward_timed.argtypes = [vp, vp, vp, vp, ct.c_int32, ct.c_int32, ct.c_int32,
                                           ct.POINTER(ct.c_double)]
        L.chf_rz_forward_graph.restype = ct.c_int
        L.chf_rz_forward_graph.argtypes = [vp, vp, vp, vp]
        L.chf_rz_sync.restype = ct.c_int
        L.chf_rz_sync.argtypes = [vp, vp]
        L.chf_rz_get_field.restype = ct.c_int
        L.chf_rz_get_field.argtypes = [vp, vp, ct.c_int32, vp]
        L.chf_rz_set_field.restype = ct.c_int
        L.chf_rz_set_field.argtypes = [vp, vp, ct.c_int32, vp]
        L.chf_rz_get_info.restype = ct.c_int
        L.chf_rz_get_info.argtypes = [vp, ct.POINTER(RZInfo)]
        L.chf_spectrum.restype = ct.c_int
        L.chf_spectrum.argtypes = [vp, vp, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_double, ct.c_double, vp,
                                   ct.c_int32, vp]
        L.chf_spectrum_project.restype = ct.c_int
        L.chf_spectrum_project.argtypes = [vp, vp, ct.c_int32, ct.c_int32, ct.c_int32, vp, vp, vp]
        L.chf_geometry_rz.restype = ct.c_int
        L.chf_geometry_rz.argtypes = [ct.c_int32, dp, ct.c_double, dp, dp]
        L.chf_geometry_xyz.restype = ct.c_int
        L.chf_geometry_xyz.argtypes = [ct.c_int32, dp, ct.c_double, ct.c_double, ct.c_double, dp, dp]
        L.chf_far_field_1d.restype = ct.c_int
        L.chf_far_field_1d.argtypes = [vp, vp, ct.c_int32, ct.c_double, ct.c_double, vp, ct.c_int32,
                                       ct.POINTER(FarFieldParams), vp, ct.c_int32, vp]
        _lib = L
        return L


def check(code: int, where: str):
    if code != CHF_OK:
        raise ChfError(code, where, lib().chf_last_error().decode(errors="replace"))
