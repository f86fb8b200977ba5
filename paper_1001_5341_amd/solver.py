"""Python face of libchfdtd: descriptors from a Workload, device memory and streams from torch.

Every numerical step runs in the HIP library; this module only marshals arguments,
allocates the caller-owned workspace and output tensors, and picks the stream.
"""
from __future__ import annotations

import ctypes as ct
import math
from typing import Optional, Sequence

import numpy as np
import torch

from . import _native as N


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def descriptors(w, storage="fp32", kernel="auto", rows=0, waves=0, zchunk=0, nan_watch=False,
                scale_e=0.0, scale_h=0.0, q_bins=None, dynamic_scaling=False):
    """Build the C descriptor structs for a workload.  Returns (structs, keepalive)."""
    q = np.ascontiguousarray(w.q_bins if q_bins is None else q_bins, dtype=np.float64)
    obs = np.ascontiguousarray(w.obs_xyz, dtype=np.float64).reshape(-1, 3)
    g = N.Grid(w.nx, w.ny, w.nz, w.n_steps, w.dx, w.dy, w.dz, w.dt)
    m = N.Medium(w.eps_r, w.mu_r, w.sigma)
    b = N.Boundary(N.BC[w.bc], w.npml if w.bc == "cpml" else 0, w.pml_m, w.pml_sigma_scale,
                   w.pml_kappa_max, w.pml_alpha_max)
    s = N.Source(w.x_axis, w.y_axis, w.z_entry, w.t_entry, w.beta, w.sigma_r, w.sigma_z,
                 w.cut_sigmas, len(q) if w.src_on else 0, 0, w.z_bin0, w.dz_bin, _dp(q))
    o = N.Observers(obs.shape[0], 0, _dp(obs))
    e = N.Exec(N.STORAGE[storage], N.KERNEL[kernel], rows, waves, zchunk, 1 if nan_watch else 0,
               scale_e, scale_h, 1 if dynamic_scaling else 0, 0)
    return (g, m, b, s, o, e), (q, obs)


def create_plan_handle(w, **kw) -> ct.c_void_p:
    """chf_plan_create only (host-side validation and tables; no device call)."""
    (g, m, b, s, o, e), keep = descriptors(w, **kw)
    h = ct.c_void_p()
    N.check(N.lib().chf_plan_create(ct.byref(g), ct.byref(m), ct.byref(b), ct.byref(s), ct.byref(o),
                                    ct.byref(e), ct.byref(h)), "chf_plan_create")
    return h


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


class Plan:
    """One shower on one grid, with its caller-owned device workspace.

    >>> plan = Plan(workload)           # validates, builds tables, binds a torch workspace
    >>> w = plan.run()                  # FP64 waveforms [n_obs, 3, n_steps] on the device
    """

    def __init__(self, w, storage: str = "fp32", kernel: str = "auto", rows: int = 0, waves: int = 0,
                 zchunk: int = 0, nan_watch: bool = False, scale_e: float = 0.0, scale_h: float = 0.0,
                 device=None, dynamic_scaling: bool = False):
        self.w = w
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.storage = storage
        # execution choices, reused by the second plan of checkpointed recomputations
        self.exec_kw = dict(kernel=kernel, rows=rows, waves=waves, zchunk=zchunk, scale_e=scale_e,
                            scale_h=scale_h, dynamic_scaling=dynamic_scaling)
        self._h = create_plan_handle(w, storage=storage, kernel=kernel, rows=rows, waves=waves,
                                     zchunk=zchunk, nan_watch=nan_watch, scale_e=scale_e,
                                     scale_h=scale_h, dynamic_scaling=dynamic_scaling)
        L = N.lib()
        nbytes = ct.c_uint64()
        N.check(L.chf_plan_workspace_bytes(self._h, ct.byref(nbytes)), "chf_plan_workspace_bytes")
        self.workspace_bytes = int(nbytes.value)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            N.check(L.chf_plan_bind_workspace(self._h, ct.c_void_p(self.workspace.data_ptr()),
                                              self.workspace_bytes, _stream_handle()),
                    "chf_plan_bind_workspace")
        self.n_obs = w.n_obs
        self.n_steps = w.n_steps

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            N.lib().chf_plan_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- info
    def info(self) -> dict:
        pi = N.PlanInfo()
        N.check(N.lib().chf_plan_get_info(self._h, ct.byref(pi)), "chf_plan_get_info")
        return {f: getattr(pi, f) for f, _ in N.PlanInfo._fields_}

    # -- running
    def new_waveforms(self) -> torch.Tensor:
        return torch.zeros((self.n_obs, 3, self.n_steps), dtype=torch.float64, device=self.device)

    def reset(self, stream=None):
        N.check(N.lib().chf_plan_reset(self._h, _stream_handle(stream)), "chf_plan_reset")

    def forward(self, n_steps: int, out: Optional[torch.Tensor] = None, first_column: int = 0,
                q_bins: Optional[torch.Tensor] = None, stream=None):
        """Advance n_steps from the current state, writing waveform columns first_column... of
        out ([n_obs, 3, ld] FP64 on the device)."""
        ld = out.shape[2] if out is not None else 0
        if out is not None:
            assert out.dtype == torch.float64 and out.is_contiguous() and out.device == self.device
        qp = ct.c_void_p(q_bins.data_ptr()) if q_bins is not None else ct.c_void_p()
        if q_bins is not None:
            assert q_bins.dtype == torch.float64 and q_bins.numel() == len(self.w.q_bins)
        wp = ct.c_void_p(out.data_ptr()) if out is not None else ct.c_void_p()
        N.check(N.lib().chf_forward(self._h, _stream_handle(stream), qp, wp, n_steps, first_column, ld),
                "chf_forward")

    def forward_timed(self, n_steps: int, out: Optional[torch.Tensor] = None, first_column: int = 0,
                      stream=None) -> float:
        """chf_forward plus hipEvents around every fused-sweep launch; returns their summed ms."""
        ld = out.shape[2] if out is not None else 0
        wp = ct.c_void_p(out.data_ptr()) if out is not None else ct.c_void_p()
        ms = ct.c_double()
        N.check(N.lib().chf_forward_timed(self._h, _stream_handle(stream), ct.c_void_p(), wp, n_steps,
                                          first_column, ld, ct.byref(ms)), "chf_forward_timed")
        return float(ms.value)

    def run(self, q_bins: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
            graph: bool = False, stream=None, sync: bool = True) -> torch.Tensor:
        """Full run from zero fields; returns [n_obs, 3, n_steps] FP64 waveforms."""
        out = self.new_waveforms() if out is None else out
        assert out.dtype == torch.float64 and out.is_contiguous() and out.device == self.device
        assert tuple(out.shape) == (self.n_obs, 3, self.n_steps)
        if q_bins is not None:
            assert q_bins.dtype == torch.float64 and q_bins.is_contiguous() and q_bins.device == self.device
            assert q_bins.numel() == len(self.w.q_bins), (q_bins.numel(), len(self.w.q_bins))
        qp = ct.c_void_p(q_bins.data_ptr()) if q_bins is not None else ct.c_void_p()
        if graph:
            N.check(N.lib().chf_forward_graph(self._h, _stream_handle(stream), qp,
                                              ct.c_void_p(out.data_ptr())), "chf_forward_graph")
        else:
            self.reset(stream)
            self.forward(self.n_steps, out, 0, q_bins, stream)
        if sync:
            self.sync(stream)
        return out

    def run_scratch(self, q_bins: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                    stream=None, sync: bool = True) -> torch.Tensor:
        """Full run from zero fields through chf_forward_scratch: inside the library's static
        device array instead of this plan's workspace (which it leaves untouched)."""
        out = self.new_waveforms() if out is None else out
        assert out.dtype == torch.float64 and out.is_contiguous() and out.device == self.device
        assert tuple(out.shape) == (self.n_obs, 3, self.n_steps)
        if q_bins is not None:
            assert q_bins.dtype == torch.float64 and q_bins.numel() == len(self.w.q_bins)
        qp = ct.c_void_p(q_bins.data_ptr()) if q_bins is not None else ct.c_void_p()
        N.check(N.lib().chf_forward_scratch(self._h, _stream_handle(stream), qp, ct.c_void_p(out.data_ptr())),
                "chf_forward_scratch")
        if sync:
            self.sync(stream)
        return out

    def sync(self, stream=None):
        N.check(N.lib().chf_plan_sync(self._h, _stream_handle(stream)), "chf_plan_sync")

    def adjoint(self, dl_dw: torch.Tensor, stream=None) -> torch.Tensor:
        assert dl_dw.dtype == torch.float64 and dl_dw.shape == (self.n_obs, 3, self.n_steps)
        dl_dw = dl_dw.contiguous()
        out = torch.zeros(len(self.w.q_bins), dtype=torch.float64, device=self.device)
        N.check(N.lib().chf_adjoint(self._h, _stream_handle(stream), ct.c_void_p(dl_dw.data_ptr()),
                                    ct.c_void_p(out.data_ptr())), "chf_adjoint")
        return out

    def adjoint_source_params(self, dl_dw: torch.Tensor, q_bins: Optional[torch.Tensor] = None, stream=None):
        """(dL/dq [n_bins], dL/dtheta [2] = (dL/dsigma_r, dL/dz_entry)) for dL/dw of the plan's full
        run (chf_adjoint_source_params)."""
        assert dl_dw.dtype == torch.float64 and dl_dw.shape == (self.n_obs, 3, self.n_steps)
        dl_dw = dl_dw.contiguous()
        dq = torch.zeros(len(self.w.q_bins), dtype=torch.float64, device=self.device)
        dth = torch.zeros(2, dtype=torch.float64, device=self.device)
        qp = ct.c_void_p(q_bins.data_ptr()) if q_bins is not None else ct.c_void_p()
        N.check(N.lib().chf_adjoint_source_params(self._h, _stream_handle(stream), ct.c_void_p(dl_dw.data_ptr()),
                                                  qp, ct.c_void_p(dq.data_ptr()), ct.c_void_p(dth.data_ptr())),
                "chf_adjoint_source_params")
        self.sync(stream)
        return dq, dth

    def adjoint_begin(self, dl_dq: torch.Tensor, stream=None):
        N.check(N.lib().chf_adjoint_begin(self._h, _stream_handle(stream), ct.c_void_p(dl_dq.data_ptr())),
                "chf_adjoint_begin")

    def adjoint_steps(self, dl_dw: torch.Tensor, dl_dq: torch.Tensor, t_lo: int, t_hi: int, stream=None):
        N.check(N.lib().chf_adjoint_steps(self._h, _stream_handle(stream), ct.c_void_p(dl_dw.data_ptr()),
                                          ct.c_void_p(dl_dq.data_ptr()), t_lo, t_hi), "chf_adjoint_steps")

    def adjoint_steps_eps(self, dl_dw: torch.Tensor, dl_dq: torch.Tensor, t_lo: int, t_hi: int,
                          e_levels: torch.Tensor, dl_deps: torch.Tensor, stream=None):
        """adjoint_steps that also accumulates dL/deps_r per E node into dl_deps ([3, nz, ny, nx]
        FP64) from the forward levels e_levels ([t_hi - t_lo + 1, 3, nz, ny, nx] FP32, level m =
        E after t_lo + m steps)."""
        w = self.w
        assert e_levels.dtype == torch.float32 and e_levels.is_contiguous()
        assert tuple(e_levels.shape) == (t_hi - t_lo + 1, 3, w.nz, w.ny, w.nx)
        assert dl_deps.dtype == torch.float64 and dl_deps.is_contiguous()
        assert tuple(dl_deps.shape) == (3, w.nz, w.ny, w.nx)
        N.check(N.lib().chf_adjoint_steps_eps(self._h, _stream_handle(stream), ct.c_void_p(dl_dw.data_ptr()),
                                              ct.c_void_p(dl_dq.data_ptr()), t_lo, t_hi,
                                              ct.c_void_p(e_levels.data_ptr()), ct.c_void_p(dl_deps.data_ptr())),
                "chf_adjoint_steps_eps")

    # -- snapshots of the whole field + CPML state
    def state_bytes(self) -> int:
        n = ct.c_uint64()
        N.check(N.lib().chf_plan_state_bytes(self._h, ct.byref(n)), "chf_plan_state_bytes")
        return int(n.value)

    def save_state(self, dst: torch.Tensor, stream=None) -> int:
        assert dst.dtype == torch.uint8 and dst.is_contiguous() and dst.numel() >= self.state_bytes()
        step = ct.c_int32()
        N.check(N.lib().chf_plan_save_state(self._h, _stream_handle(stream), ct.c_void_p(dst.data_ptr()),
                                            ct.byref(step)), "chf_plan_save_state")
        return int(step.value)

    def load_state(self, src: torch.Tensor, step: int, stream=None):
        assert src.dtype == torch.uint8 and src.is_contiguous() and src.numel() >= self.state_bytes()
        N.check(N.lib().chf_plan_load_state(self._h, _stream_handle(stream), ct.c_void_p(src.data_ptr()), step),
                "chf_plan_load_state")

    # -- field access (physical units, [nz, ny, nx] FP32)
    def get_field(self, comp: int, stream=None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Component 0..5 = Ex, Ey, Ez, Hx, Hy, Hz of the current level as [nz, ny, nx] FP32
        (physical units), into `out` when given (contiguous FP32 of that shape)."""
        if out is None:
            out = torch.empty((self.w.nz, self.w.ny, self.w.nx), dtype=torch.float32, device=self.device)
        assert out.dtype == torch.float32 and out.is_contiguous()
        assert tuple(out.shape) == (self.w.nz, self.w.ny, self.w.nx)
        N.check(N.lib().chf_plan_get_field(self._h, _stream_handle(stream), comp,
                                           ct.c_void_p(out.data_ptr())), "chf_plan_get_field")
        return out

    def set_field(self, comp: int, value: torch.Tensor, stream=None):
        v = value.to(device=self.device, dtype=torch.float32).contiguous()
        assert v.shape == (self.w.nz, self.w.ny, self.w.nx)
        N.check(N.lib().chf_plan_set_field(self._h, _stream_handle(stream), comp,
                                           ct.c_void_p(v.data_ptr())), "chf_plan_set_field")
        torch.cuda.current_stream().synchronize()


def run(w, **kw) -> torch.Tensor:
    """One-shot forward run of a workload; returns device FP64 waveforms [n_obs, 3, n_steps]."""
    plan = Plan(w, **kw)
    try:
        return plan.run()
    finally:
        plan.close()


class Batch:
    """Several plans advanced together: one launch per phase per step for the whole batch,
    the whole run captured once into a hipGraph (chf_batch_run)."""

    def __init__(self, plans: Sequence[Plan]):
        self.plans = list(plans)
        arr = (ct.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        self._keep = arr
        self._h = ct.c_void_p()
        L = N.lib()
        N.check(L.chf_batch_create(len(self.plans), arr, ct.byref(self._h)), "chf_batch_create")
        nbytes = ct.c_uint64()
        N.check(L.chf_batch_workspace_bytes(self._h, ct.byref(nbytes)), "chf_batch_workspace_bytes")
        dev = self.plans[0].device
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=dev)
        N.check(L.chf_batch_bind_workspace(self._h, ct.c_void_p(self.workspace.data_ptr()), int(nbytes.value),
                                           _stream_handle()), "chf_batch_bind_workspace")

    def run(self, outs=None, stream=None, sync=True, persistent=False):
        """The whole batch run from zero fields: one captured graph of per-phase launches, or
        (persistent=True) one cooperative kernel launch looping over the steps."""
        outs = outs or [p.new_waveforms() for p in self.plans]
        ptrs = (ct.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        self._ptrs = ptrs
        fn = "chf_batch_run_persistent" if persistent else "chf_batch_run"
        N.check(getattr(N.lib(), fn)(self._h, _stream_handle(stream), ptrs), fn)
        if sync:
            for p in self.plans:
                p.sync(stream)
        return outs

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            N.lib().chf_batch_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def checkpointed_adjoint(plan: "Plan", dl_dw: torch.Tensor, every: Optional[int] = None,
                         verify: bool = True, q_bins: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """dL/dq by checkpointed recomputation: a forward run on a second workspace keeps a
    snapshot every `every` steps (default ceil(sqrt(T))); the reverse sweep then takes the
    segments last to first, restores each segment's snapshot, recomputes its forward steps
    (with the profile q_bins the forward run used, default the plan's)
    and applies the transposed steps of that segment to the adjoint state.

    verify=False runs the whole schedule in the library (chf_adjoint_checkpointed).  verify=True
    drives the same schedule from here through the step-range entry points and checks that every
    recomputed segment ends on the next snapshot bit for bit (a determinism check).

    The profile map is linear with zero initial fields, so the transposed steps do not read
    the recomputed forward states: the result is bitwise that of Plan.adjoint.  The schedule
    is the one gradients with respect to non-linear parameters need (eps_sensitivity)."""
    T = plan.n_steps
    K = max(1, min(T, every or math.ceil(math.sqrt(T))))
    n_seg = (T + K - 1) // K
    fwd = Plan(plan.w, storage=plan.storage, device=plan.device, **plan.exec_kw)
    try:
        nbytes = fwd.state_bytes()
        snaps = torch.empty((n_seg, nbytes), dtype=torch.uint8, device=plan.device)
        dl_dw = dl_dw.to(torch.float64).contiguous()
        dq = torch.zeros(len(plan.w.q_bins), dtype=torch.float64, device=plan.device)
        if not verify:
            q = ct.c_void_p(q_bins.data_ptr()) if q_bins is not None else ct.c_void_p()
            N.check(N.lib().chf_adjoint_checkpointed(
                plan._h, fwd._h, _stream_handle(stream), q, ct.c_void_p(dl_dw.data_ptr()),
                ct.c_void_p(dq.data_ptr()), K, ct.c_void_p(snaps.data_ptr()), snaps.numel(), ct.c_void_p(),
                ct.c_void_p()), "chf_adjoint_checkpointed")
            plan.sync(stream)
            return dq
        fwd.reset(stream)
        for s_ in range(n_seg):
            fwd.save_state(snaps[s_], stream)
            fwd.forward(min(K, T - s_ * K), None, 0, q_bins, stream)
        tail = torch.empty(nbytes, dtype=torch.uint8, device=plan.device)
        plan.adjoint_begin(dq, stream)
        for s_ in reversed(range(n_seg)):
            t0, t1 = s_ * K, min((s_ + 1) * K, T)
            fwd.load_state(snaps[s_], t0, stream)
            fwd.forward(t1 - t0, None, 0, q_bins, stream)
            if s_ + 1 < n_seg:
                fwd.save_state(tail, stream)
                if not torch.equal(tail, snaps[s_ + 1]):
                    raise RuntimeError(f"recomputed segment {s_} does not reproduce its snapshot")
            plan.adjoint_steps(dl_dw, dq, t0, t1, stream)
        plan.sync(stream)
        return dq
    finally:
        fwd.close()


def eps_sensitivity(plan: "Plan", dl_dw: torch.Tensor, every: Optional[int] = None,
                    q_bins: Optional[torch.Tensor] = None, stream=None):
    """dL/deps_r at every E node (the gradient with respect to a relative-permittivity map,
    evaluated at the plan's uniform medium) and dL/dq, for L = <dl_dw, w>.

    The permittivity is a non-linear parameter: its cotangent at step n reads the forward
    levels E^n and E^{n+1}, which come back in reverse order by checkpointed recomputation
    (chf_adjoint_checkpointed): a forward run on a second workspace keeps a snapshot every
    `every` steps (default ceil(sqrt(T))); the reverse sweep takes the segments last to first,
    restores a segment's snapshot, recomputes its steps one by one keeping the E levels
    (every + 1 levels of 3 nx ny nz FP32 values), and runs that segment's transposed steps with
    the permittivity term.  Returns (dl_deps [3, nz, ny, nx] FP64, dl_dq [n_bins] FP64); for a
    uniform medium with PEC walls, dL/deps_r of the plan is dl_deps.sum()."""
    w = plan.w
    T = plan.n_steps
    K = max(1, min(T, every or math.ceil(math.sqrt(T))))
    n_seg = (T + K - 1) // K
    fwd = Plan(w, storage=plan.storage, device=plan.device, **plan.exec_kw)
    try:
        snaps = torch.empty((n_seg, fwd.state_bytes()), dtype=torch.uint8, device=plan.device)
        dl_dw = dl_dw.to(torch.float64).contiguous()
        dq = torch.zeros(len(w.q_bins), dtype=torch.float64, device=plan.device)
        g = torch.zeros((3, w.nz, w.ny, w.nx), dtype=torch.float64, device=plan.device)
        levels = torch.empty((K + 1, 3, w.nz, w.ny, w.nx), dtype=torch.float32, device=plan.device)
        q = ct.c_void_p(q_bins.data_ptr()) if q_bins is not None else ct.c_void_p()
        N.check(N.lib().chf_adjoint_checkpointed(
            plan._h, fwd._h, _stream_handle(stream), q, ct.c_void_p(dl_dw.data_ptr()), ct.c_void_p(dq.data_ptr()),
            K, ct.c_void_p(snaps.data_ptr()), snaps.numel(), ct.c_void_p(levels.data_ptr()),
            ct.c_void_p(g.data_ptr())), "chf_adjoint_checkpointed")
        plan.sync(stream)
        return g, dq
    finally:
        fwd.close()


class CherenkovFDTD(torch.autograd.Function):
    """Waveforms as a differentiable function of the longitudinal profile bins.

    forward:  w = A q  (the full run from zero fields; FP64 waveforms [n_obs, 3, n_steps])
    backward: dL/dq = A^T dL/dw by the library's discrete adjoint (exact transpose of the
              forward recurrence run backward in time), in one reverse sweep by default.
              With checkpoint_every it runs the checkpointed schedule instead
              (checkpointed_adjoint): same bits, but for this linear map the recomputed forward
              states are not read, so that schedule only costs time here; it is the one the
              permittivity gradient (eps_sensitivity) needs.
    The gradient comes back on the input's device and in its dtype."""

    @staticmethod
    def forward(ctx, q_bins: torch.Tensor, plan: "Plan", checkpoint_every: Optional[int] = None):
        if q_bins.numel() != len(plan.w.q_bins):
            raise ValueError(f"q_bins has {q_bins.numel()} entries, the plan's profile {len(plan.w.q_bins)}")
        ctx.plan = plan
        ctx.every = checkpoint_every
        ctx.in_device, ctx.in_dtype, ctx.in_shape = q_bins.device, q_bins.dtype, q_bins.shape
        q = q_bins.detach().to(device=plan.device, dtype=torch.float64).contiguous().reshape(-1)
        ctx.q = q
        return plan.run(q_bins=q)

    @staticmethod
    def backward(ctx, grad_w: torch.Tensor):
        g = grad_w.to(device=ctx.plan.device, dtype=torch.float64).contiguous()
        if ctx.every:
            dq = checkpointed_adjoint(ctx.plan, g, every=ctx.every, q_bins=ctx.q)
        else:
            dq = ctx.plan.adjoint(g)
            ctx.plan.sync()
        return dq.reshape(ctx.in_shape).to(device=ctx.in_device, dtype=ctx.in_dtype), None, None


def waveforms(q_bins: torch.Tensor, plan: "Plan", checkpoint_every: Optional[int] = None) -> torch.Tensor:
    return CherenkovFDTD.apply(q_bins, plan, checkpoint_every)


# ---------------------------------------------------------------- axisymmetric (r, z) solver
def rz_descriptors(w, vx=0, waves=0, zchunk=0, nan_watch=False, q_bins=None, steps_per_launch=0,
                   storage="fp32", dynamic_scaling=False, scale_e=0.0, scale_h=0.0):
    """C descriptor structs for an RZWorkload.  Returns (structs, keepalive)."""
    q = np.ascontiguousarray(w.q_bins if q_bins is None else q_bins, dtype=np.float64)
    obs = np.ascontiguousarray(w.obs_rz, dtype=np.float64).reshape(-1, 2)
    g = N.RZGrid(w.nr, w.nz, w.n_steps, 0, w.dr, w.dz, w.dt)
    m = N.Medium(w.eps_r, w.mu_r, w.sigma)
    s = N.RZSource(w.z_entry, w.t_entry, w.beta, w.sigma_r, w.sigma_z, w.cut_sigmas,
                   len(q) if w.src_on else 0, 0, w.z_bin0, w.dz_bin, _dp(q))
    o = N.RZObservers(obs.shape[0], 0, _dp(obs))
    e = N.RZExec(N.BC[w.bc], vx, waves, zchunk, 1 if nan_watch else 0, steps_per_launch, N.STORAGE[storage],
                 1 if dynamic_scaling else 0, scale_e, scale_h)
    return (g, m, s, o, e), (q, obs)


def create_rz_plan_handle(w, **kw) -> ct.c_void_p:
    """chf_rz_plan_create only (host-side validation and tables; no device call)."""
    (g, m, s, o, e), keep = rz_descriptors(w, **kw)
    h = ct.c_void_p()
    N.check(N.lib().chf_rz_plan_create(ct.byref(g), ct.byref(m), ct.byref(s), ct.byref(o), ct.byref(e),
                                       ct.byref(h)), "chf_rz_plan_create")
    return h


class RZPlan:
    """The axisymmetric solver on one (r, z) grid, with its caller-owned device workspace.

    >>> plan = RZPlan(rz_workload)
    >>> w = plan.run()                  # FP64 waveforms [n_obs, 2 (E_r, E_z), n_steps]
    """

    def __init__(self, w, vx: int = 0, waves: int = 0, zchunk: int = 0, nan_watch: bool = False,
                 steps_per_launch: int = 0, storage: str = "fp32", dynamic_scaling: bool = False,
                 scale_e: float = 0.0, scale_h: float = 0.0, device=None):
        self.w = w
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._h = create_rz_plan_handle(w, vx=vx, waves=waves, zchunk=zchunk, nan_watch=nan_watch,
                                        steps_per_launch=steps_per_launch, storage=storage,
                                        dynamic_scaling=dynamic_scaling, scale_e=scale_e, scale_h=scale_h)
        self.storage = storage
        L = N.lib()
        nbytes = ct.c_uint64()
        N.check(L.chf_rz_workspace_bytes(self._h, ct.byref(nbytes)), "chf_rz_workspace_bytes")
        self.workspace_bytes = int(nbytes.value)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            N.check(L.chf_rz_bind_workspace(self._h, ct.c_void_p(self.workspace.data_ptr()),
                                            self.workspace_bytes, _stream_handle()), "chf_rz_bind_workspace")
        self.n_obs = w.n_obs
        self.n_steps = w.n_steps

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            N.lib().chf_rz_plan_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        ri = N.RZInfo()
        N.check(N.lib().chf_rz_get_info(self._h, ct.byref(ri)), "chf_rz_get_info")
        return {f: getattr(ri, f) for f, _ in N.RZInfo._fields_}

    def new_waveforms(self) -> torch.Tensor:
        return torch.zeros((self.n_obs, 2, self.n_steps), dtype=torch.float64, device=self.device)

    def reset(self, stream=None):
        N.check(N.lib().chf_rz_reset(self._h, _stream_handle(stream)), "chf_rz_reset")

    @staticmethod
    def _ptr(t: Optional[torch.Tensor]) -> ct.c_void_p:
        return ct.c_void_p(t.data_ptr()) if t is not None else ct.c_void_p()

    def _check_io(self, out, q_bins):
        if out is not None:
            assert out.dtype == torch.float64 and out.is_contiguous() and out.device == self.device
            assert out.shape[:2] == (self.n_obs, 2)
        if q_bins is not None:
            assert q_bins.dtype == torch.float64 and q_bins.numel() == len(self.w.q_bins)

    def forward(self, n_steps: int, out: Optional[torch.Tensor] = None, first_column: int = 0,
                q_bins: Optional[torch.Tensor] = None, stream=None):
        self._check_io(out, q_bins)
        ld = out.shape[2] if out is not None else 0
        N.check(N.lib().chf_rz_forward(self._h, _stream_handle(stream), self._ptr(q_bins), self._ptr(out),
                                       n_steps, first_column, ld), "chf_rz_forward")

    def forward_timed(self, n_steps: int, out: Optional[torch.Tensor] = None, first_column: int = 0,
                      stream=None) -> float:
        """chf_rz_forward plus hipEvents around every sweep launch; returns their summed ms."""
        self._check_io(out, None)
        ld = out.shape[2] if out is not None else 0
        ms = ct.c_double()
        N.check(N.lib().chf_rz_forward_timed(self._h, _stream_handle(stream), ct.c_void_p(), self._ptr(out),
                                             n_steps, first_column, ld, ct.byref(ms)), "chf_rz_forward_timed")
        return float(ms.value)

    def run(self, q_bins: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
            graph: bool = False, stream=None, sync: bool = True) -> torch.Tensor:
        """Full run from zero fields; returns [n_obs, 2, n_steps] FP64 waveforms."""
        out = self.new_waveforms() if out is None else out
        self._check_io(out, q_bins)
        if graph:
            N.check(N.lib().chf_rz_forward_graph(self._h, _stream_handle(stream), self._ptr(q_bins),
                                                 self._ptr(out)), "chf_rz_forward_graph")
        else:
            self.reset(stream)
            self.forward(self.n_steps, out, 0, q_bins, stream)
        if sync:
            self.sync(stream)
        return out

    def sync(self, stream=None):
        N.check(N.lib().chf_rz_sync(self._h, _stream_handle(stream)), "chf_rz_sync")

    def get_field(self, comp: int, stream=None) -> torch.Tensor:
        """Component 0 = E_r, 1 = E_z, 2 = H_phi of the current level as [nz, nr] FP32."""
        out = torch.empty((self.w.nz, self.w.nr), dtype=torch.float32, device=self.device)
        N.check(N.lib().chf_rz_get_field(self._h, _stream_handle(stream), comp, ct.c_void_p(out.data_ptr())),
                "chf_rz_get_field")
        return out

    def set_field(self, comp: int, value: torch.Tensor, stream=None):
        v = value.to(device=self.device, dtype=torch.float32).contiguous()
        assert v.shape == (self.w.nz, self.w.nr)
        N.check(N.lib().chf_rz_set_field(self._h, _stream_handle(stream), comp, ct.c_void_p(v.data_ptr())),
                "chf_rz_set_field")
        torch.cuda.current_stream().synchronize()
