"""FP64 oracle for the paper's own axisymmetric scheme (TEST INFRASTRUCTURE ONLY).

What it computes (Numerical Method section, eqs. fdtd_Er, fdtd_Ez, fdtd_Hphi): with cylindrical
symmetry about the shower axis only E_r, E_z and H_phi survive, and the curl equations become

    eps dE_r/dt + sigma E_r = -dH_phi/dz
    eps dE_z/dt + sigma E_z = (1/r) d(r H_phi)/dr  - J_z
    mu dH_phi/dt            = dE_z/dr - dE_r/dz

discretised with central differences on the (r, z) restriction of the Yee lattice and the
leapfrog in time: nodes r_i = i dr (i = 0..nr-1), z_k = k dz; E_r(i+1/2, k), E_z(i, k+1/2),
H_phi(i+1/2, k+1/2); E at n dt, H at (n+1/2) dt.  Readings (the paper gives the equations
only): the shower current enters eq. fdtd_Ez as in the 3-D scheme; on the axis the radial
term is Stokes' theorem over the disc of radius dr/2, i.e. the same discrete divergence
with the cell "radius" of the axis cell taken as dr/8 (area pi dr^2/4 per 2 pi dr); the wall
at r_max and the z walls are PEC or first-order Mur on the tangential E; the radial charge
weights are Gaussians normalised on the lattice with the ring areas of the E_z cells.

It shares no code with the HIP path.  Arrays are [z, r].
"""
from __future__ import annotations

import math

import numpy as np

C0 = 299_792_458.0
MU0 = 1.25663706212e-6  # CODATA 2018
EPS0 = 1.0 / (MU0 * C0 * C0)


def ring_radius(nr: int, dr: float) -> np.ndarray:
    """Per-radian area factor of the E_z cells (area = 2 pi * factor * dr): r_i for i >= 1,
    dr/8 on the axis (a disc of radius dr/2)."""
    a = np.arange(nr) * dr
    a[0] = dr / 8.0
    return a


class RZState:
    def __init__(self, w, q_bins=None):
        self.w = w
        self.q = np.asarray(w.q_bins if q_bins is None else q_bins, dtype=np.float64)
        nr, nz = w.nr, w.nz
        self.er = np.zeros((nz, nr))  # E_r(i+1/2, k): i <= nr-2
        self.ez = np.zeros((nz, nr))  # E_z(i, k+1/2): k <= nz-2
        self.hp = np.zeros((nz, nr))  # H_phi(i+1/2, k+1/2): i <= nr-2, k <= nz-2
        eps, mu = EPS0 * w.eps_r, MU0 * w.mu_r
        loss = w.sigma * w.dt / (2.0 * eps)
        self.ca = (1.0 - loss) / (1.0 + loss)
        self.cb = (w.dt / eps) / (1.0 + loss)
        self.db = w.dt / mu
        self.rz_cell = ring_radius(nr, w.dr)                 # E_z nodes
        self.rh = (np.arange(nr) + 0.5) * w.dr               # H_phi nodes r_{i+1/2}
        self.n = 0
        # radial charge weights on the E_z nodes (the wall node excluded), sum W * 2 pi a dr = 1
        r = np.arange(nr) * w.dr
        g = np.where((r <= w.cut_sigmas * w.sigma_r) & (np.arange(nr) <= nr - 2),
                     np.exp(-0.5 * (r / w.sigma_r) ** 2), 0.0)
        self.wr = g / (g * 2.0 * math.pi * self.rz_cell * w.dr).sum() if w.src_on else g * 0.0
        self._observers()

    # -- source (the same moving bunch as in 3-D, on the axis)
    def charge(self, z: float) -> float:
        """Q(z) from the hat-function bins of the longitudinal profile."""
        u = (z - self.w.z_bin0) / self.w.dz_bin
        b = math.floor(u)
        t = u - b
        q = 0.0
        if 0 <= b < len(self.q):
            q += (1.0 - t) * self.q[b]
        if 0 <= b + 1 < len(self.q):
            q += t * self.q[b + 1]
        return q

    def current_z(self, n: int) -> np.ndarray:
        """J_z at (n+1/2) dt (Simulation Setup section: the charge excess moving along the axis
        at beta c0): v Q(z_s) times the z weights (a Gaussian in z sampled at the E_z rows of its
        window, normalised to unit integral) times the radial weights."""
        w = self.w
        jz = np.zeros((w.nz, w.nr))
        t = (n + 0.5) * w.dt
        if not w.src_on or t < w.t_entry:
            return jz
        v = w.beta * C0
        zs = w.z_entry + v * (t - w.t_entry)
        half = w.cut_sigmas * w.sigma_z
        ks = np.arange(math.ceil((zs - half) / w.dz - 0.5), math.floor((zs + half) / w.dz - 0.5) + 1)
        wz = np.exp(-0.5 * (((ks + 0.5) * w.dz - zs) / w.sigma_z) ** 2)
        wz = wz / (wz.sum() * w.dz)
        keep = (ks >= 0) & (ks <= w.nz - 2)
        jz[ks[keep]] = v * self.charge(zs) * wz[keep][:, None] * self.wr[None, :]
        return jz

    # -- updates
    def update_h(self):
        """Eq. fdtd_Hphi: mu dH_phi/dt = dE_z/dr - dE_r/dz, central differences."""
        w = self.w
        dez_dr = (self.ez[:-1, 1:] - self.ez[:-1, :-1]) / w.dr
        der_dz = (self.er[1:, :-1] - self.er[:-1, :-1]) / w.dz
        self.hp[:-1, :-1] += self.db * (dez_dr - der_dz)

    def update_e(self):
        """Eqs. fdtd_Er and fdtd_Ez with sigma (semi-implicit), then the boundary."""
        w = self.w
        old = (self.er.copy(), self.ez.copy()) if w.bc == "mur1" else None
        jz = self.current_z(self.n)
        # E_r(i+1/2, k), 1 <= k <= nz-2, i <= nr-2
        dh_dz = (self.hp[1:-1, :-1] - self.hp[:-2, :-1]) / w.dz
        self.er[1:-1, :-1] = self.ca * self.er[1:-1, :-1] - self.cb * dh_dz
        # E_z(i, k+1/2), i <= nr-2 (the axis included), k <= nz-2
        flux = self.rh[None, :-1] * self.hp[:-1, :-1]           # r_{i+1/2} H(i+1/2)
        inner = np.zeros_like(flux)
        inner[:, 1:] = flux[:, :-1]                             # r_{i-1/2} H(i-1/2); 0 on the axis
        div = (flux - inner) / (self.rz_cell[None, :-1] * w.dr)
        self.ez[:-1, :-1] = self.ca * self.ez[:-1, :-1] + self.cb * (div - jz[:-1, :-1])
        if old is not None:
            self._mur(*old)
        self.n += 1

    def _mur(self, er_old, ez_old):
        """First-order Mur on the tangential E: E_z at r_max (k <= nz-2), E_r at the z walls
        (i <= nr-2)."""
        w = self.w
        v = C0 / math.sqrt(w.eps_r * w.mu_r)

        def k(d):
            return (v * w.dt - d) / (v * w.dt + d)

        kr, kz = k(w.dr), k(w.dz)
        nr, nz = w.nr, w.nz
        self.ez[:-1, nr - 1] = ez_old[:-1, nr - 2] + kr * (self.ez[:-1, nr - 2] - ez_old[:-1, nr - 1])
        self.er[0, :-1] = er_old[1, :-1] + kz * (self.er[1, :-1] - er_old[0, :-1])
        self.er[nz - 1, :-1] = er_old[nz - 2, :-1] + kz * (self.er[nz - 2, :-1] - er_old[nz - 1, :-1])

    # -- observers: bilinear on each component's sub-lattice
    def _observers(self):
        w = self.w
        self.stencils = []
        for r, z in np.asarray(w.obs_rz, dtype=np.float64).reshape(-1, 2):
            comps = []
            for c in range(2):  # 0: E_r at (i+1/2, k); 1: E_z at (i, k+1/2)
                fr = r / w.dr - (0.5 if c == 0 else 0.0)
                fz = z / w.dz - (0.5 if c == 1 else 0.0)
                i0, k0 = math.floor(fr), math.floor(fz)
                comps.append((i0, k0, fr - i0, fz - k0))
            self.stencils.append(comps)

    def sample(self) -> np.ndarray:
        out = np.zeros((len(self.stencils), 2))
        for o, comps in enumerate(self.stencils):
            for c, (i0, k0, tr, tz) in enumerate(comps):
                f = self.er if c == 0 else self.ez
                out[o, c] = ((1 - tz) * ((1 - tr) * f[k0, i0] + tr * f[k0, i0 + 1])
                             + tz * ((1 - tr) * f[k0 + 1, i0] + tr * f[k0 + 1, i0 + 1]))
        return out

    def step(self) -> np.ndarray:
        self.update_h()
        self.update_e()
        return self.sample()


def run(w, q_bins=None) -> np.ndarray:
    """Waveforms [n_obs][2][n_steps] (E_r, E_z); column n is E at (n+1) dt."""
    st = RZState(w, q_bins)
    out = np.zeros((len(st.stencils), 2, w.n_steps))
    for n in range(w.n_steps):
        out[:, :, n] = st.step()
    return out
