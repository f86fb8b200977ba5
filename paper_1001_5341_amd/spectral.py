"""Spectral and angular post-processing of recorded pulses (include/chfdtd_spectral.h).

E_omega spectra of the waveforms (FP64 DFT kernel), their theta-hat component and modulus,
observer geometry (R, theta from the shower maximum), and the far-field formula of the paper's
Comparison section (eq. 1d_appro) for the same charge profile, all through the library; this
module marshals arguments and arranges results.  `power_law_exponent` is host-side reporting
over kernel outputs (a log-log slope across a handful of distances).
"""
from __future__ import annotations

import ctypes as ct
from typing import Optional

import numpy as np
import torch

from . import _native as N


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def _dev_f64(x, device) -> torch.Tensor:
    t = torch.as_tensor(x, dtype=torch.float64, device=device)
    return t.contiguous()


def spectrum(waves: torch.Tensor, dt: float, omega, t0: Optional[float] = None, stream=None) -> torch.Tensor:
    """E(omega) of waveforms [..., n_t] (FP64 on the device; column n is time t0 + n dt, default
    t0 = dt as the solvers record E^{n+1}) -> complex128 [..., n_freq]."""
    assert waves.dtype == torch.float64 and waves.is_cuda
    lead = waves.shape[:-1]
    n_t = waves.shape[-1]
    w = waves.reshape(-1, n_t).contiguous()
    om = _dev_f64(omega, waves.device).reshape(-1)
    out = torch.empty((w.shape[0], om.numel(), 2), dtype=torch.float64, device=waves.device)
    N.check(N.lib().chf_spectrum(_stream(stream), ct.c_void_p(w.data_ptr()), w.shape[0], n_t, n_t, dt,
                                 dt if t0 is None else t0, ct.c_void_p(om.data_ptr()), om.numel(),
                                 ct.c_void_p(out.data_ptr())), "chf_spectrum")
    return torch.view_as_complex(out).reshape(*lead, om.numel())


def project(spec: torch.Tensor, weights, stream=None):
    """Component spectra [n_obs, n_comp, n_freq] (complex128) and weights [n_obs, n_comp] ->
    (complex projection [n_obs, n_freq], modulus [n_obs, n_freq])."""
    n_obs, n_comp, n_freq = spec.shape
    s = torch.view_as_real(spec.contiguous()).contiguous()
    wts = _dev_f64(weights, spec.device).reshape(n_obs, n_comp)
    out = torch.empty((n_obs, n_freq, 2), dtype=torch.float64, device=spec.device)
    mag = torch.empty((n_obs, n_freq), dtype=torch.float64, device=spec.device)
    N.check(N.lib().chf_spectrum_project(_stream(stream), ct.c_void_p(s.data_ptr()), n_obs, n_comp, n_freq,
                                         ct.c_void_p(wts.data_ptr()), ct.c_void_p(out.data_ptr()),
                                         ct.c_void_p(mag.data_ptr())), "chf_spectrum_project")
    return torch.view_as_complex(out), mag


def geometry(w):
    """(r_theta [n_obs, 2], theta-hat weights [n_obs, n_comp]) of a workload's observers seen from
    its shower maximum on the axis (host arrays)."""
    L = N.lib()
    if hasattr(w, "obs_rz"):
        obs = np.ascontiguousarray(w.obs_rz, dtype=np.float64).reshape(-1, 2)
        rt = np.zeros((obs.shape[0], 2))
        wts = np.zeros((obs.shape[0], 2))
        N.check(L.chf_geometry_rz(obs.shape[0], _dp(obs), w.z_origin, _dp(rt), _dp(wts)), "chf_geometry_rz")
    else:
        obs = np.ascontiguousarray(w.obs_xyz, dtype=np.float64).reshape(-1, 3)
        rt = np.zeros((obs.shape[0], 2))
        wts = np.zeros((obs.shape[0], 3))
        N.check(L.chf_geometry_xyz(obs.shape[0], _dp(obs), w.x_axis, w.y_axis, w.z_origin, _dp(rt), _dp(wts)),
                "chf_geometry_xyz")
    return rt, wts


def far_field(w, r_theta, omega, q_bins=None, device=None, stream=None) -> torch.Tensor:
    """E_theta(omega) of the far-field formula for the workload's profile and medium at the given
    (R, theta) pairs -> complex128 [n_obs, n_freq] on the device."""
    device = device or torch.device("cuda", torch.cuda.current_device())
    q = _dev_f64(w.q_bins if q_bins is None else q_bins, device)
    rt = _dev_f64(r_theta, device).reshape(-1, 2)
    om = _dev_f64(omega, device).reshape(-1)
    out = torch.empty((rt.shape[0], om.numel(), 2), dtype=torch.float64, device=device)
    prm = N.FarFieldParams(float(np.sqrt(w.eps_r * w.mu_r)), w.beta, w.z_entry, w.t_entry, w.z_origin)
    N.check(N.lib().chf_far_field_1d(_stream(stream), ct.c_void_p(q.data_ptr()), q.numel(), w.z_bin0, w.dz_bin,
                                     ct.c_void_p(rt.data_ptr()), rt.shape[0], ct.byref(prm),
                                     ct.c_void_p(om.data_ptr()), om.numel(), ct.c_void_p(out.data_ptr())),
            "chf_far_field_1d")
    return torch.view_as_complex(out)


def theta_spectra(w, waves: torch.Tensor, omega, stream=None):
    """Everything for the Results-section plots of one run: (r_theta, E_theta(omega) complex,
    |E_theta(omega)|, far-field |E_theta(omega)|), all [n_obs, n_freq] except r_theta."""
    rt, wts = geometry(w)
    spec = spectrum(waves, w.dt, omega, stream=stream)
    e_th, mag = project(spec, wts, stream=stream)
    ff = far_field(w, rt, omega, device=waves.device, stream=stream)
    return rt, e_th, mag, ff.abs()


def power_law_exponent(R, mag) -> np.ndarray:
    """Least-squares slope of ln|E| against ln R for each frequency (columns of mag [n_R, n_f]):
    -1/2 for a cylindrical wave, -1 for a spherical one."""
    x = np.log(np.asarray(R, dtype=np.float64))
    y = np.log(np.asarray(mag, dtype=np.float64))
    xm = x - x.mean()
    return (xm[:, None] * (y - y.mean(axis=0))).sum(axis=0) / (xm * xm).sum()
