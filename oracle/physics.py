"""Continuum physics references used to pin the FP64 oracle (test infrastructure only).

* Field of a point electric dipole p(t) z^ in a uniform medium (near, intermediate and
  radiation terms, retarded time t - r/v): the time-domain form of the Green's-function
  solution the paper starts from (Coherent Cherenkov Pulses section, vector potential
  integral), for a single current element.
* The superposition of such dipoles for a whole sampled current distribution J_z(x, t) on a
  set of points: the continuum field of that distribution (static, induction and radiation
  terms), against which the lattice's propagation of the same source is checked.
* Fraunhofer spectrum of a line current (the paper's far-field approximation) and the
  closed form of the 1-D far-field formula for a Gaussian profile (Comparison section).
* Cherenkov cone geometry: cos(theta_c) = 1/(n beta), which is where the paper's phase
  p = (1 - n cos theta) omega / c vanishes, and the first-arrival time of the shock front.
"""
from __future__ import annotations

import math

import numpy as np

C0 = 299_792_458.0
MU0 = 1.25663706212e-6
EPS0 = 1.0 / (MU0 * C0 * C0)


def dipole_e_field(r_vec, t, p, pd, pdd, eps_r: float, mu_r: float = 1.0):
    """E(r, t) of a z-directed point dipole with moment p(t) (callables for p, dp/dt, d2p/dt2).

    E = 1/(4 pi eps) [ (3 r^(r^.p) - p)/r^3 + (3 r^(r^.p') - p')/(v r^2)
                       + (r^(r^.p'') - p'')/(v^2 r) ]  at the retarded time t - r/v.
    r_vec: (3,) displacement from the dipole; t: array of times.  Returns (len(t), 3)."""
    eps = EPS0 * eps_r
    v = C0 / math.sqrt(eps_r * mu_r)
    r_vec = np.asarray(r_vec, dtype=np.float64)
    r = float(np.linalg.norm(r_vec))
    rh = r_vec / r
    z = np.array([0.0, 0.0, 1.0])
    tr = np.asarray(t, dtype=np.float64) - r / v
    P, PD, PDD = p(tr), pd(tr), pdd(tr)
    a = 3.0 * rh * rh[2] - z          # (3 r^(r^.z) - z)
    b = rh * rh[2] - z                # (r^(r^.z) - z)
    E = (np.outer(P, a) / r ** 3 + np.outer(PD, a) / (v * r ** 2) + np.outer(PDD, b) / (v * v * r))
    return E / (4.0 * math.pi * eps)


def dipole_superposition(pos, pdot_half, dt: float, obs, t_out, eps_r: float, mu_r: float = 1.0):
    """E at observers from z-directed point dipoles at `pos` (M, 3) whose moment derivatives
    dp/dt (= J_z dV, A m) are sampled at the half steps (n + 1/2) dt, n = 0..T-1 (pdot_half (M, T);
    zero before).  Each dipole's moment at the integer steps is p_n = dt sum_{m<n} pdot_{m+1/2},
    dp/dt there the mean of the neighbouring half steps, d2p/dt2 their difference over dt; the
    three are interpolated linearly in time at the retarded time t - r/v and put into the
    dipole field (near, intermediate and radiation terms).  obs: (n_obs, 3); t_out: times.
    Returns (n_obs, 3, len(t_out))."""
    eps = EPS0 * eps_r
    v = C0 / math.sqrt(eps_r * mu_r)
    pos = np.asarray(pos, dtype=np.float64)
    M, T = pdot_half.shape
    zero = np.zeros((M, 1))
    p_int = np.concatenate([zero, np.cumsum(pdot_half, axis=1) * dt], axis=1)          # n = 0..T
    pdp = np.concatenate([zero, pdot_half, zero], axis=1)                              # n -1/2 .. T+1/2
    pd_int = 0.5 * (pdp[:, :-1] + pdp[:, 1:])
    pdd_int = (pdp[:, 1:] - pdp[:, :-1]) / dt
    t_out = np.asarray(t_out, dtype=np.float64)
    out = np.zeros((len(obs), 3, len(t_out)))
    for o, ob in enumerate(np.asarray(obs, dtype=np.float64)):
        rv = ob[None, :] - pos
        r = np.linalg.norm(rv, axis=1)
        rh = rv / r[:, None]
        s = (t_out[None, :] - (r / v)[:, None]) / dt
        i0 = np.clip(np.floor(s).astype(np.int64), 0, T - 1)
        f = np.clip(s - i0, 0.0, 1.0)
        valid = s >= 0

        def at(a):
            x = np.take_along_axis(a, i0, axis=1) * (1 - f) + np.take_along_axis(a, i0 + 1, axis=1) * f
            return np.where(valid, x, 0.0)

        P, PD, PDD = at(p_int), at(pd_int), at(pdd_int)
        for c in range(3):
            zc = 1.0 if c == 2 else 0.0
            a_c = 3.0 * rh[:, c] * rh[:, 2] - zc
            b_c = rh[:, c] * rh[:, 2] - zc
            E = (P * (a_c / r ** 3)[:, None] + PD * (a_c / (v * r ** 2))[:, None]
                 + PDD * (b_c / (v * v * r))[:, None])
            out[o, c] = E.sum(axis=0) / (4.0 * math.pi * eps)
    return out


def lowpass(x, dt: float, fc: float):
    """Gaussian low-pass exp(-(f/fc)^2) along the last axis, the record extended by its edge
    values on both sides (so that a static tail does not wrap round)."""
    n = x.shape[-1]
    padn = 4 * n
    xp = np.pad(x, [(0, 0)] * (x.ndim - 1) + [(n, padn - 2 * n)], mode="edge")
    X = np.fft.rfft(xp, axis=-1)
    X *= np.exp(-(np.fft.rfftfreq(padn, dt) / fc) ** 2)
    return np.fft.irfft(X, padn, axis=-1)[..., n:2 * n]


def gaussian_dipole(p0: float, t0: float, tau: float):
    """p(t) = p0 exp(-(t-t0)^2 / (2 tau^2)) and its first two derivatives."""
    def p(t):
        return p0 * np.exp(-0.5 * ((t - t0) / tau) ** 2)

    def pd(t):
        return -p0 * (t - t0) / tau ** 2 * np.exp(-0.5 * ((t - t0) / tau) ** 2)

    def pdd(t):
        u = (t - t0) / tau
        return p0 / tau ** 2 * (u * u - 1.0) * np.exp(-0.5 * u * u)

    return p, pd, pdd


def cherenkov_angle(n: float, beta: float = 1.0) -> float:
    return math.acos(1.0 / (n * beta))


def shock_arrival_time(rho: float, z_obs: float, z_entry: float, n: float, beta: float = 1.0,
                       t_entry: float = 0.0) -> float:
    """First arrival of the Cherenkov front at (rho, z_obs) for a charge entering at z_entry at
    t_entry and moving at beta c0: minimise t(z') = (z'-z_entry)/v + n |x - x'|/c0 over z'."""
    v = beta * C0
    return t_entry + (z_obs - z_entry) / v + rho * math.sqrt(n * n * beta * beta - 1.0) / (beta * C0)


def fraunhofer_line_spectrum(omega, theta: float, R: float, z_prime, current_fn, n: float,
                             t_grid):
    """Far-field E_theta(omega) of a z-directed current I(z', t) on the axis, using the
    Fraunhofer phase exp(ikR - ik x^.x') of the paper:
      A_w = mu/(4 pi R) e^{ikR} sum_z' dz' int dt e^{i w t} I(z',t) e^{-ik cos(theta) z'},
      E_perp = i w A_w sin(theta)  (magnitude of the transverse part).
    current_fn(z', t) -> I (ampere).  Returns complex array over omega."""
    omega = np.atleast_1d(np.asarray(omega, dtype=np.float64))
    z_prime = np.asarray(z_prime, dtype=np.float64)
    t_grid = np.asarray(t_grid, dtype=np.float64)
    dzp = z_prime[1] - z_prime[0]
    dt = t_grid[1] - t_grid[0]
    k = omega * n / C0
    out = np.zeros(len(omega), dtype=np.complex128)
    I = np.array([current_fn(zp, t_grid) for zp in z_prime])  # (nz', nt)
    for m, (w, kk) in enumerate(zip(omega, k)):
        tw = np.exp(1j * w * t_grid) * dt
        Iw = I @ tw                                    # (nz',)
        out[m] = np.sum(Iw * np.exp(-1j * kk * math.cos(theta) * z_prime)) * dzp
    A = MU0 / (4.0 * math.pi * R) * np.exp(1j * k * R) * out
    return 1j * omega * A * math.sin(theta)


def gaussian_profile_far_field(omega, theta: float, R: float, n_max_charge: float, length: float,
                               n: float, beta: float = 1.0):
    """The paper's 1-D formula for a Gaussian longitudinal profile N_max exp(-z^2/2l^2) moving
    at v = beta c0 (charge per particle folded into n_max_charge, coulomb):
      E = sqrt(2 pi) e/(4 pi eps0 c^2) i w sin(theta) e^{ikR}/R N_max l exp(-l^2 p^2/2),
      p = (1/beta - n cos theta) w / c0   (p = (1 - n cos theta) w/c at beta = 1).
    Written with mu0 = 1/(eps0 c^2).  Sign convention: E(w) = int dt e^{+i w t} E(t)."""
    omega = np.atleast_1d(np.asarray(omega, dtype=np.float64))
    k = omega * n / C0
    p = (1.0 / beta - n * math.cos(theta)) * omega / C0
    amp = math.sqrt(2.0 * math.pi) * MU0 / (4.0 * math.pi) * n_max_charge * length
    return 1j * omega * math.sin(theta) * np.exp(1j * k * R) / R * amp * np.exp(-0.5 * (length * p) ** 2)
