"""Pins of the spectral oracle against what the mathematics fixes: numpy's FFT at its own
frequencies, the analytic transform of a Gaussian pulse, the closed-form far field of a Gaussian
profile (eq. 1d_appro) and of a single hat bin, and the geometry of the polarisation vector."""
import math

import numpy as np
import pytest

from oracle import physics as ph
from oracle import spectral_oracle as S


def test_dft_equals_inverse_fft_at_its_frequencies():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 256))
    dt = 2.5e-11
    om = 2 * math.pi * np.arange(256) / (256 * dt)
    got = S.dft(x, dt, 0.0, om)
    want = dt * 256 * np.fft.ifft(x, axis=-1)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_dft_of_gaussian_pulse_matches_analytic_transform():
    tau, tc, dt = 0.3e-9, 4e-9, 0.02e-9
    n = 500
    t0 = dt
    t = t0 + dt * np.arange(n)
    x = np.exp(-0.5 * ((t - tc) / tau) ** 2)
    om = 2 * math.pi * np.linspace(0, 1.5e9, 31)
    got = S.dft(x, dt, t0, om)
    want = tau * math.sqrt(2 * math.pi) * np.exp(-0.5 * (om * tau) ** 2) * np.exp(1j * om * tc)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * abs(want[0]))


def test_single_hat_bin_transform_closed_form():
    h, zb = 0.07, 1.3
    p = np.linspace(-60, 60, 41)
    got = S.profile_transform([2.0], zb, h, p, sub=4096)  # trapezoid error (p h/sub)^2/12 < 1e-7
    sinc = np.where(p == 0, 1.0, np.sin(0.5 * p * h) / np.where(p == 0, 1, 0.5 * p * h))
    want = 2.0 * h * sinc ** 2 * np.exp(1j * p * zb)
    np.testing.assert_allclose(got, want, rtol=0, atol=2e-7 * 2.0 * h)


@pytest.mark.parametrize("theta_deg", [40.0, 55.0, 70.0])
def test_far_field_of_gaussian_profile_matches_eq_1d_appro(theta_deg):
    """Fine hat bins of N exp(-(z - zc)^2/2l^2) against the closed form, magnitudes and phases
    (the closed form puts the profile centre at z = 0: the phase e^{i p zc} is removed)."""
    n_idx, l, zc, nmax = 1.78, 0.8, 5.0, -1e-10
    h = 0.01
    zb = np.arange(0.0, 10.0 + h / 2, h)  # +-6.25 l: truncation below 1e-8
    q = nmax * np.exp(-0.5 * ((zb - zc) / l) ** 2)
    th = math.radians(theta_deg)
    om = 2 * math.pi * np.array([5e6, 50e6, 100e6, 300e6, 600e6])
    R = 40.0
    got = S.far_field_theta(q, 0.0, h, [R], [th], n_idx, 1.0, om)[0]
    p = (1.0 - n_idx * math.cos(th)) * om / S.C0
    got = got * np.exp(-1j * p * zc)
    want = -ph.gaussian_profile_far_field(om, th, R, nmax, l, n_idx)
    ok = np.abs(want) > 1e-4 * np.abs(want).max()
    # hat interpolation changes the transform by sinc^2(p h/2) ~ 1 - (p h)^2/12 (< 2e-4 here)
    np.testing.assert_allclose(got[ok], want[ok], rtol=3e-4)


def test_far_field_vanishes_along_the_axis_and_peaks_on_the_cone():
    n_idx, h = 1.78, 0.01
    zb = np.arange(0.0, 4.0, h)
    q = -1e-10 * np.exp(-0.5 * ((zb - 2.0) / 0.5) ** 2)
    om = np.array([2 * math.pi * 300e6])
    th = np.radians(np.linspace(0.0, 90.0, 181))
    e = np.abs(S.far_field_theta(q, 0.0, h, np.full(th.size, 30.0), th, n_idx, 1.0, om))[:, 0]
    assert e[0] == 0.0
    # without the sin(theta) of the transverse projection the profile factor peaks where the
    # phase p = (1 - n cos theta) w / c vanishes: on the Cherenkov cone
    f = e[1:] / np.sin(th[1:])
    assert abs(th[1:][np.argmax(f)] - math.acos(1 / n_idx)) <= math.radians(0.5)


def test_theta_projection_geometry():
    z0 = 2.0
    obs = np.array([[3.0, 2.0 + 4.0], [1.0, 2.0 - 1.0], [2.0, 2.0]])
    R, th = S.geometry_rz(obs, z0)
    np.testing.assert_allclose(R, [5.0, math.sqrt(2.0), 2.0])
    wts = S.theta_weights_rz(obs, z0)
    # a field along R-hat has no theta component; one along theta-hat has unit component
    rhat = np.stack([np.sin(th), np.cos(th)], 1)
    that = np.stack([np.cos(th), -np.sin(th)], 1)
    np.testing.assert_allclose((wts * rhat).sum(1), 0.0, atol=1e-15)
    np.testing.assert_allclose((wts * that).sum(1), 1.0)
    # the 3-D weights at phi = 0 reduce to the (r, z) ones
    obs3 = np.stack([10.0 + obs[:, 0], np.full(3, 7.0), obs[:, 1]], 1)
    w3 = S.theta_weights_xyz(obs3, 10.0, 7.0, z0)
    np.testing.assert_allclose(w3[:, [0, 2]], wts, atol=1e-15)
    np.testing.assert_allclose(w3[:, 1], 0.0, atol=1e-15)
