"""FP64 oracle of the spectral post-processing (TEST INFRASTRUCTURE ONLY).

What it computes (Results section: E_omega spectra at fixed R and theta, their scaling with R
and their angular distribution; Comparison section: the 1-D far-field formula, eq. 1d_appro):

* the spectrum of a recorded waveform, E(omega) = int E(t) exp(+i omega t) dt, as the rectangle
  rule over the samples, sum_n E(t0 + n dt) exp(i omega (t0 + n dt)) dt (the sign convention of
  the paper's Green's-function integral, eq. GreenMethod);
* the polarisation component along theta-hat (the direction n_perp of eq. 1d_appro) at an
  observer seen from the origin (the axis point at the shower maximum), R and theta measured
  from there (the paper's spherical detector coordinates);
* the far-field spectrum of the moving charge profile: with the Fraunhofer phase (eq. fraun_appr)
  the vector potential of the bunch, whose centre passes z' at t'(z') = t_entry + (z' - z_entry)/v,
  is A_z = mu0/(4 pi) e^{ikR}/R e^{i omega t_off} e^{ik cos(theta) z_o} F(p),
  F(p) = int Q(z') e^{i p z'} dz', p = omega/v - k cos(theta), t_off = t_entry - z_entry/v,
  and E_theta = -i omega sin(theta) A_z (the transverse part of i omega A).  For beta = 1 this is
  eq. 1d_appro with e N_e(z') = Q(z').  F is integrated numerically here (dense sampling of
  the hat-interpolated profile), not by its closed form.

Plain NumPy; it shares no code with the HIP path.
"""
from __future__ import annotations

import math

import numpy as np

C0 = 299_792_458.0
MU0 = 1.25663706212e-6


def dft(w: np.ndarray, dt: float, t0: float, omega: np.ndarray) -> np.ndarray:
    """[..., n_t] real samples at t0 + n dt -> [..., n_freq] complex spectra."""
    w = np.asarray(w, dtype=np.float64)
    t = t0 + dt * np.arange(w.shape[-1])
    ker = np.exp(1j * np.outer(t, np.asarray(omega, dtype=np.float64))) * dt
    return w @ ker


def geometry_rz(obs_rz: np.ndarray, z_origin: float):
    """R and theta of (r, z) observers seen from the axis point z_origin."""
    obs = np.asarray(obs_rz, dtype=np.float64).reshape(-1, 2)
    r, dz = obs[:, 0], obs[:, 1] - z_origin
    return np.hypot(r, dz), np.arctan2(r, dz)


def theta_weights_rz(obs_rz: np.ndarray, z_origin: float) -> np.ndarray:
    """E_theta = E . theta-hat with theta-hat = cos(theta) r-hat - sin(theta) z-hat: weights on
    (E_r, E_z) per observer, [n_obs, 2]."""
    _, th = geometry_rz(obs_rz, z_origin)
    return np.stack([np.cos(th), -np.sin(th)], axis=1)


def geometry_xyz(obs_xyz: np.ndarray, x_axis: float, y_axis: float, z_origin: float):
    obs = np.asarray(obs_xyz, dtype=np.float64).reshape(-1, 3)
    dx, dy, dz = obs[:, 0] - x_axis, obs[:, 1] - y_axis, obs[:, 2] - z_origin
    rho = np.hypot(dx, dy)
    return np.sqrt(rho * rho + dz * dz), np.arctan2(rho, dz), np.arctan2(dy, dx)


def theta_weights_xyz(obs_xyz, x_axis, y_axis, z_origin) -> np.ndarray:
    """theta-hat = (cos(theta) cos(phi), cos(theta) sin(phi), -sin(theta)), [n_obs, 3]."""
    _, th, ph = geometry_xyz(obs_xyz, x_axis, y_axis, z_origin)
    return np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], axis=1)


def project(spec: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """[n_obs, n_comp, n_freq] spectra and [n_obs, n_comp] weights -> [n_obs, n_freq]."""
    return np.einsum("ocf,oc->of", spec, weights)


def hat_profile(z: np.ndarray, q_bins, z_bin0: float, dz_bin: float) -> np.ndarray:
    """Q(z) = sum_b q_b hat((z - z_bin0)/dz_bin - b): linear between bin nodes, zero one bin
    beyond each end."""
    q = np.concatenate([[0.0], np.asarray(q_bins, dtype=np.float64), [0.0]])
    nodes = z_bin0 + dz_bin * np.arange(-1, len(q) - 1)
    return np.interp(z, nodes, q, left=0.0, right=0.0)


def profile_transform(q_bins, z_bin0: float, dz_bin: float, p: np.ndarray, sub: int = 64) -> np.ndarray:
    """F(p) = int Q(z) e^{i p z} dz by the trapezoid rule on `sub` points per bin (exact up to
    O((p dz_bin / sub)^2) on the piecewise-linear Q)."""
    n = len(q_bins)
    z = z_bin0 + dz_bin * (np.arange((n + 1) * sub + 1) / sub - 1.0)
    qz = hat_profile(z, q_bins, z_bin0, dz_bin)
    h = dz_bin / sub
    wts = np.full(len(z), h)
    wts[0] = wts[-1] = 0.5 * h
    p = np.atleast_1d(np.asarray(p, dtype=np.float64))
    return np.exp(1j * np.outer(p, z)) @ (qz * wts)


def far_field_theta(q_bins, z_bin0: float, dz_bin: float, R, theta, n_index: float, beta: float,
                    omega, z_entry: float = 0.0, t_entry: float = 0.0, z_origin: float = 0.0,
                    sub: int = 64) -> np.ndarray:
    """E_theta(omega) of the far-field formula for each (R, theta) pair: [n_obs, n_freq]."""
    R = np.atleast_1d(np.asarray(R, dtype=np.float64))
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    omega = np.atleast_1d(np.asarray(omega, dtype=np.float64))
    v = beta * C0
    k = n_index * omega / C0
    t_off = t_entry - z_entry / v
    out = np.zeros((len(R), len(omega)), dtype=np.complex128)
    for o in range(len(R)):
        p = omega / v - k * math.cos(theta[o])
        F = profile_transform(q_bins, z_bin0, dz_bin, p, sub)
        A = MU0 / (4.0 * math.pi) * np.exp(1j * k * R[o]) / R[o] * np.exp(1j * omega * t_off) \
            * np.exp(1j * k * math.cos(theta[o]) * z_origin) * F
        out[o] = -1j * omega * math.sin(theta[o]) * A
    return out
