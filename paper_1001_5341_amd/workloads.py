"""Seeded synthetic workloads: grid, medium, boundary, shower profile and observers.

This module only *generates inputs*; it holds none of the solver's arithmetic (no
update coefficients, no source weights, no CPML grading, no interpolation).  Both
the HIP path and the FP64 oracle consume the ``Workload`` objects built here.

Physical inputs follow the paper's Simulation Setup section:
  * the longitudinal development is either a Gaussian N_max exp(-z^2/2l^2)
    (the Gaussian fit of the NKG formula) or a Greisen-type profile
    exp[t (1 - 1.5 ln s)] with age s = 3t/(t + 2 t_max) (the NKG/Greisen
    parametrisation, with the commonly quoted form of the age), stretched so that
    its RMS length is the drawn shower length;
  * the shower moves along +z; the detector geometry is spherical, centred where
    the shower axis crosses the shower maximum, with observers placed by (R, theta).
The charge excess is negative (knocked-on electrons), so Q0 < 0.

Every random quantity comes from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import math
from typing import List, Optional

import numpy as np

C0 = 299_792_458.0  # m/s, exact
N_ICE = 1.78


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    n_steps: int
    dx: float
    dy: float
    dz: float
    dt: float
    eps_r: float = N_ICE ** 2
    mu_r: float = 1.0
    sigma: float = 0.0
    bc: str = "cpml"  # "pec" | "mur1" | "cpml"
    npml: int = 10
    pml_m: float = 3.0
    pml_sigma_scale: float = 1.0
    pml_kappa_max: float = 1.0
    pml_alpha_max: float = 0.0
    src_on: bool = True
    x_axis: float = 0.0
    y_axis: float = 0.0
    z_entry: float = 0.0
    t_entry: float = 0.0
    beta: float = 1.0
    sigma_r: float = 0.02
    sigma_z: float = 0.01
    cut_sigmas: float = 4.0
    z_bin0: float = 0.0
    dz_bin: float = 0.01
    q_bins: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(2))
    obs_xyz: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3)))
    seed: int = 0
    notes: str = ""
    z_origin: float = 0.0  # axis point the observers' (R, theta) are measured from (shower maximum)

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_obs(self) -> int:
        return int(self.obs_xyz.shape[0])

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)

    def describe(self) -> dict:
        return {
            "workload": self.name, "grid": [self.nx, self.ny, self.nz], "steps": self.n_steps,
            "dx_m": self.dx, "dt_s": self.dt, "bc": self.bc, "npml": self.npml,
            "n_obs": self.n_obs, "n_bins": int(len(self.q_bins)), "seed": self.seed,
        }


def courant_dt(dx: float, dy: float, dz: float, frac: float = 0.99) -> float:
    """dt = frac * dx / (c0 sqrt 3) for a cubic lattice (the vacuum Courant limit)."""
    return frac / (C0 * math.sqrt(1.0 / dx ** 2 + 1.0 / dy ** 2 + 1.0 / dz ** 2))


def draw_q0(rng: np.random.Generator) -> float:
    """Charge-excess scale in coulomb: Q0 = -10^U(-12,-9)."""
    return -(10.0 ** rng.uniform(-12.0, -9.0))


def cherenkov_theta(n: float = N_ICE, beta: float = 1.0) -> float:
    """Observer placement only: the cone half-angle arccos(1/(n beta))."""
    return math.acos(1.0 / (n * beta))


def greisen_shape(t: np.ndarray, t_max: float = 10.0) -> np.ndarray:
    """exp[t (1 - 1.5 ln s)], s = 3t/(t + 2 t_max), zero for t <= 0 (maximum at t = t_max)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    pos = t > 0
    tp = t[pos]
    s = 3.0 * tp / (tp + 2.0 * t_max)
    out[pos] = np.exp(tp * (1.0 - 1.5 * np.log(s)))
    return out


def _greisen_rms(t_max: float = 10.0) -> float:
    t = np.linspace(1e-6, 8 * t_max, 200_001)
    f = greisen_shape(t, t_max)
    m0 = f.sum()
    mu = (t * f).sum() / m0
    return math.sqrt(((t - mu) ** 2 * f).sum() / m0)


def _taper(z: np.ndarray, z0: float, z1: float, ramp: float) -> np.ndarray:
    """cos^2 ramps to zero at z0 and z1 so that the charge appears and disappears smoothly."""
    w = np.ones_like(z)
    w[(z <= z0) | (z >= z1)] = 0.0
    a = (z > z0) & (z < z0 + ramp)
    w[a] = np.sin(0.5 * math.pi * (z[a] - z0) / ramp) ** 2
    b = (z < z1) & (z > z1 - ramp)
    w[b] = np.sin(0.5 * math.pi * (z1 - z[b]) / ramp) ** 2
    return w


def greisen_profile_bins(z_bins: np.ndarray, z_max: float, length: float, q0: float,
                         z_on: float, z_off: float, ramp: float, t_max: float = 10.0) -> np.ndarray:
    lam = length / _greisen_rms(t_max)
    t = t_max + (z_bins - z_max) / lam
    f = greisen_shape(t, t_max) / greisen_shape(np.array([t_max]), t_max)[0]
    return q0 * f * _taper(z_bins, z_on, z_off, ramp)


def place_observers(rng: np.random.Generator, n_obs: int, origin, lo, hi,
                    r_min: float, r_max: float, theta_deg=(40.0, 70.0)) -> np.ndarray:
    """theta ~ U[theta_deg], phi ~ U[0, 2pi), R ~ U[r_min, min(r_max, R_fit)], where R_fit
    keeps the point inside the box [lo, hi] (each a 3-vector)."""
    origin = np.asarray(origin, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    out = []
    tries = 0
    while len(out) < n_obs:
        tries += 1
        if tries > 100000:
            raise RuntimeError("cannot place observers in this grid")
        th = math.radians(rng.uniform(*theta_deg))
        ph = rng.uniform(0.0, 2.0 * math.pi)
        d = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        r_fit = np.inf
        for u in range(3):
            if d[u] > 1e-12:
                r_fit = min(r_fit, (hi[u] - origin[u]) / d[u])
            elif d[u] < -1e-12:
                r_fit = min(r_fit, (lo[u] - origin[u]) / d[u])
        top = min(r_max, r_fit)
        if top < r_min:
            continue
        r = rng.uniform(r_min, top)
        out.append(origin + r * d)
    return np.array(out, dtype=np.float64)


def _interior_box(nx, ny, nz, dx, dy, dz, margin_cells):
    lo = np.array([margin_cells * dx, margin_cells * dy, margin_cells * dz])
    hi = np.array([(nx - 1 - margin_cells) * dx, (ny - 1 - margin_cells) * dy,
                   (nz - 1 - margin_cells) * dz])
    return lo, hi


def gaussian_cube(seed: int = 1, n: int = 64, n_steps: int = 400, bc: str = "mur1",
                  name: Optional[str] = None) -> Workload:
    """Plain 64^3 case: Gaussian Q(z)=Q0 exp(-(z-z0)^2/(2*0.15 m^2)) on 1 mm bins, line charge at
    v = c along z with a 2 cm Gaussian radial width, Mur boundary, 8 observers on a ring of
    diameter 0.5 m on the Cherenkov cone."""
    rng = np.random.default_rng(seed)
    d = 0.01
    L = (n - 1) * d
    z0 = 0.5 * L
    q0 = draw_q0(rng)
    dzb = 0.001
    zb = np.arange(0.0, L + 0.5 * dzb, dzb)
    q = q0 * np.exp(-((zb - z0) ** 2) / (2.0 * 0.15))
    rho = 0.25 * min(1.0, (n - 1) / 63.0)  # ring of diameter 0.5 m at 64^3, scaled below
    zo = z0 + rho / math.tan(cherenkov_theta())
    phis = np.deg2rad(45.0 * np.arange(8))
    obs = np.stack([0.5 * L + rho * np.cos(phis), 0.5 * L + rho * np.sin(phis),
                    np.full(8, zo)], axis=1)
    return Workload(name=name or f"gaussian-{n}^3", nx=n, ny=n, nz=n, n_steps=n_steps,
                    dx=d, dy=d, dz=d, dt=courant_dt(d, d, d), bc=bc, npml=10 if bc == "cpml" else 0,
                    x_axis=0.5 * L, y_axis=0.5 * L, z_entry=0.0, t_entry=0.0, beta=1.0,
                    sigma_r=0.02, sigma_z=0.01, z_bin0=0.0, dz_bin=dzb, q_bins=q, obs_xyz=obs,
                    seed=seed)


def greisen_shower(seed: int, nx: int, ny: int, nz: int, n_steps: int, n_obs: int,
                   d: float = 0.01, npml: int = 10, bc: str = "cpml", sigma_r: float = 0.03,
                   zmax_frac=None, zmax_range=(6.0, 10.0), length_range=(3.0, 8.0),
                   r_range=(1.0, 5.0), z_entry: Optional[float] = None, name: str = "",
                   alpha_max: Optional[float] = None) -> Workload:
    """Greisen-like shower on a z-elongated grid with a CPML (the single-shower, precision,
    batched and adjoint workloads).  Shower maximum and length are drawn from the seed; when
    they do not fit the grid they are scaled into it (zmax_frac gives the range as fractions
    of the z extent)."""
    rng = np.random.default_rng(seed)
    Lz = (nz - 1) * d
    if zmax_frac is not None:
        z_max = rng.uniform(*zmax_frac) * Lz
    else:
        z_max = rng.uniform(*zmax_range)
    length = rng.uniform(*length_range)
    q0 = draw_q0(rng)
    x_axis = 0.5 * (nx - 1) * d
    y_axis = 0.5 * (ny - 1) * d
    if z_entry is None:
        z_entry = (npml + 5) * d
    z_off = (nz - 1 - npml - 5) * d
    ramp = min(0.3, 0.25 * (z_off - z_entry))
    zb = np.arange(z_entry, z_off + 0.5 * d, d)
    q = greisen_profile_bins(zb, z_max, length, q0, z_entry, z_off, ramp)
    lo, hi = _interior_box(nx, ny, nz, d, d, d, npml + 3)
    origin = np.array([x_axis, y_axis, z_max])
    obs = place_observers(rng, n_obs, origin, lo, hi, r_range[0], r_range[1])
    if alpha_max is None:
        alpha_max = 2.0 * math.pi * 50e6 * 8.8541878128e-12
    return Workload(name=name or f"greisen-{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, n_steps=n_steps,
                    dx=d, dy=d, dz=d, dt=courant_dt(d, d, d), bc=bc, npml=npml if bc == "cpml" else 0,
                    pml_alpha_max=alpha_max, x_axis=x_axis, y_axis=y_axis, z_entry=z_entry,
                    t_entry=0.0, beta=1.0, sigma_r=sigma_r, sigma_z=0.01, z_bin0=float(zb[0]),
                    dz_bin=d, q_bins=q, obs_xyz=obs, seed=seed, z_origin=z_max,
                    notes=f"z_max={z_max:.3f} m, length={length:.3f} m, Q0={q0:.3e} C")


def single_shower(seed: int = 2) -> Workload:
    """FP32 single shower: 256x256x2048 cells of 1 cm, n=1.78, 10-cell CPML, 4000 steps,
    Greisen-like profile (shower max 6-10 m, length 3-8 m), 3 cm radial Gaussian, 64 observers
    at theta 40-70 deg and R from 1 m up to what fits the cross-section."""
    return greisen_shower(seed, 256, 256, 2048, 4000, 64, name="single-shower-256x256x2048")


def precision_shower(seed: int = 2) -> Workload:
    """Same shower as single_shower on a 512x512x4096 grid, 6000 steps."""
    w = single_shower(seed)
    big = greisen_shower(seed, 512, 512, 4096, 6000, 64, name="precision-512x512x4096")
    # same shower and the same observer offsets from the shower maximum
    off = w.obs_xyz - np.array([w.x_axis, w.y_axis, 0.0])
    obs = off + np.array([big.x_axis, big.y_axis, 0.0])
    zb = np.arange(w.z_bin0, w.z_bin0 + w.dz_bin * len(w.q_bins) - 0.5 * w.dz_bin, w.dz_bin)
    return big.replace(q_bins=w.q_bins.copy(), z_bin0=w.z_bin0, dz_bin=w.dz_bin, obs_xyz=obs,
                       z_entry=w.z_entry, z_origin=w.z_origin, notes=w.notes + f"; {len(zb)} bins")


def batch_showers(seed: int = 4, count: int = 32, n_steps: int = 2000, n_obs: int = 16) -> List[Workload]:
    """Uneven batch: n_x = n_y in {96..256}, n_z in [max(n_x,96), 1024], per-shower profile."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n = int(rng.choice([96, 128, 160, 192, 224, 256]))
        nz = int(rng.integers(max(n, 96) // 32, 1024 // 32 + 1)) * 32
        sub = int(rng.integers(0, 2 ** 31 - 1))
        r_lo = 0.2
        r_hi = 0.5 * (n - 1) * 0.01
        out.append(greisen_shower(sub, n, n, nz, n_steps, n_obs, zmax_frac=(0.3, 0.6),
                                  length_range=(0.1 * (nz - 1) * 0.01, 0.3 * (nz - 1) * 0.01),
                                  r_range=(r_lo, r_hi), name=f"batch{s}-{n}x{n}x{nz}"))
    return out


def adjoint_problem(seed_target: int = 5, seed_start: int = 6, nx: int = 128, ny: int = 128,
                    nz: int = 1024, n_steps: int = 3000, n_obs: int = 16, n_bins: int = 128,
                    npml: int = 10):
    """Differentiation workload: 128 hat bins spanning the z extent, target profile q* from one
    seed and the evaluation point q = q* + perturbation from the next.  Returns
    (workload at q, q_target)."""
    d = 0.01
    half = 0.5 * (min(nx, ny) - 1 - 2 * (npml + 3)) * d
    base = greisen_shower(seed_target, nx, ny, nz, n_steps, n_obs, npml=npml,
                          zmax_frac=(0.35, 0.55), length_range=(0.1 * nz * d, 0.25 * nz * d),
                          r_range=(min(0.3, 0.5 * half), 2.0), name=f"adjoint-{nx}x{ny}x{nz}")
    dz_bin = nz * d / n_bins
    zc = np.arange(n_bins) * dz_bin
    # sample the target profile at the bin centres
    fine_z = base.z_bin0 + base.dz_bin * np.arange(len(base.q_bins))
    q_target = np.interp(zc, fine_z, base.q_bins, left=0.0, right=0.0)
    rng = np.random.default_rng(seed_start)
    scale = np.max(np.abs(q_target)) if np.any(q_target) else 1e-10
    q = q_target + 0.2 * scale * rng.standard_normal(n_bins) * (q_target != 0)
    w = base.replace(q_bins=q, z_bin0=0.0, dz_bin=dz_bin)
    return w, q_target


def small_shower(seed: int = 11, nx: int = 72, ny: int = 60, nz: int = 150, n_steps: int = 260,
                 n_obs: int = 8, bc: str = "cpml", npml: int = 8) -> Workload:
    """Reduced shower for parity tests: several tiles per axis with ragged tails."""
    d = 0.01
    return greisen_shower(seed, nx, ny, nz, n_steps, n_obs, d=d, npml=npml if bc == "cpml" else 0,
                          bc=bc, sigma_r=0.02, zmax_frac=(0.35, 0.55),
                          length_range=(0.15 * nz * d, 0.3 * nz * d),
                          r_range=(0.12, 0.5), name=f"small-{nx}x{ny}x{nz}-{bc}")


def workload_by_name(name: str, seed: Optional[int] = None) -> Workload:
    table = {
        "gaussian-64": lambda s: gaussian_cube(1 if s is None else s),
        "single-shower": lambda s: single_shower(2 if s is None else s),
        "precision": lambda s: precision_shower(2 if s is None else s),
        "small": lambda s: small_shower(11 if s is None else s),
    }
    return table[name](seed)


def workload_digest(w) -> str:
    """SHA-256 of everything that defines a workload's inputs (stored expected values carry it)."""
    h = hashlib.sha256()
    h.update(json.dumps(w.describe(), sort_keys=True).encode())
    for arr in (w.q_bins, w.obs_xyz):
        h.update(np.ascontiguousarray(arr, dtype=np.float64).tobytes())
    for v in (w.dt, w.dx, w.x_axis, w.y_axis, w.z_entry, w.sigma_r, w.sigma_z, w.pml_alpha_max):
        h.update(np.float64(v).tobytes())
    return h.hexdigest()


# ------------------------------------------------------------ axisymmetric (r, z) workloads
@dataclasses.dataclass
class RZWorkload:
    """Inputs of the axisymmetric scheme: nr x nz nodes (node i at r = i dr, node k at
    z = k dz; the axis is node column 0 and the outer wall is column nr-1), the same moving
    shower source as in 3-D (centred on the axis), observers given as (r, z) pairs."""
    name: str
    nr: int
    nz: int
    n_steps: int
    dr: float
    dz: float
    dt: float
    eps_r: float = N_ICE ** 2
    mu_r: float = 1.0
    sigma: float = 0.0
    bc: str = "mur1"  # "pec" | "mur1"
    src_on: bool = True
    z_entry: float = 0.0
    t_entry: float = 0.0
    beta: float = 1.0
    sigma_r: float = 0.02
    sigma_z: float = 0.01
    cut_sigmas: float = 4.0
    z_bin0: float = 0.0
    dz_bin: float = 0.01
    q_bins: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(2))
    obs_rz: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 2)))
    seed: int = 0
    notes: str = ""
    z_origin: float = 0.0  # axis point the observers' (R, theta) are measured from (shower maximum)

    @property
    def n_cells(self) -> int:
        return self.nr * self.nz

    @property
    def n_obs(self) -> int:
        return int(self.obs_rz.shape[0])

    def replace(self, **kw) -> "RZWorkload":
        return dataclasses.replace(self, **kw)

    def describe(self) -> dict:
        return {
            "workload": self.name, "grid": [self.nr, self.nz], "steps": self.n_steps,
            "dr_m": self.dr, "dz_m": self.dz, "dt_s": self.dt, "bc": self.bc,
            "n_obs": self.n_obs, "n_bins": int(len(self.q_bins)), "seed": self.seed,
        }


def place_observers_rz(rng: np.random.Generator, n_obs: int, z_origin: float, r_hi: float,
                       z_lo: float, z_hi: float, r_min: float, r_max: float, r_lo: float,
                       theta_deg=(40.0, 70.0)) -> np.ndarray:
    """(R, theta) about the point (0, z_origin): theta ~ U[theta_deg], R ~ U[r_min, min(r_max,
    R_fit)], where R_fit keeps r in [r_lo, r_hi] and z in [z_lo, z_hi]."""
    out = []
    tries = 0
    while len(out) < n_obs:
        tries += 1
        if tries > 100000:
            raise RuntimeError("cannot place observers in this grid")
        th = math.radians(rng.uniform(*theta_deg))
        s, c = math.sin(th), math.cos(th)
        r_fit = r_hi / s
        if c > 1e-12:
            r_fit = min(r_fit, (z_hi - z_origin) / c)
        elif c < -1e-12:
            r_fit = min(r_fit, (z_lo - z_origin) / c)
        top = min(r_max, r_fit)
        bot = max(r_min, r_lo / s)
        if top < bot:
            continue
        R = rng.uniform(bot, top)
        out.append((R * s, z_origin + R * c))
    return np.array(out, dtype=np.float64)


def rz_shower(seed: int, nr: int, nz: int, n_steps: int, n_obs: int, d: float = 0.01,
              bc: str = "mur1", sigma_r: float = 0.03, zmax_frac=(0.2, 0.35),
              length_range=(3.0, 8.0), r_range=(1.0, 64.0), margin: int = 4,
              name: str = "") -> RZWorkload:
    """Greisen-like shower on an (r, z) grid of square cells: the axisymmetric counterpart of
    greisen_shower.  The shower enters near the lower z wall and is switched off near the upper
    one; observers at theta 40-70 deg about the shower maximum with R drawn in r_range (clipped
    to what fits the grid), at least `margin` cells from the walls and the axis."""
    rng = np.random.default_rng(seed)
    Lz = (nz - 1) * d
    z_max = rng.uniform(*zmax_frac) * Lz
    length = min(rng.uniform(*length_range), 0.25 * Lz)
    q0 = draw_q0(rng)
    z_entry = (margin + 5) * d
    z_off = (nz - 1 - margin - 5) * d
    ramp = min(0.3, 0.25 * (z_off - z_entry))
    zb = np.arange(z_entry, z_off + 0.5 * d, d)
    q = greisen_profile_bins(zb, z_max, length, q0, z_entry, z_off, ramp)
    obs = place_observers_rz(rng, n_obs, z_max, (nr - 1 - margin) * d, margin * d,
                             (nz - 1 - margin) * d, r_range[0], r_range[1], margin * d)
    return RZWorkload(name=name or f"rz-{nr}x{nz}", nr=nr, nz=nz, n_steps=n_steps, dr=d, dz=d,
                      dt=courant_dt(d, d, d), bc=bc, z_entry=z_entry, t_entry=0.0, beta=1.0,
                      sigma_r=sigma_r, sigma_z=0.01, z_bin0=float(zb[0]), dz_bin=d, q_bins=q,
                      obs_rz=obs, seed=seed, z_origin=z_max,
                      notes=f"z_max={z_max:.3f} m, length={length:.3f} m, Q0={q0:.3e} C")


def rz_small(seed: int = 21, nr: int = 300, nz: int = 520, n_steps: int = 700, n_obs: int = 12,
             bc: str = "mur1") -> RZWorkload:
    """Reduced (r, z) shower for parity tests: several tiles in r and z with ragged tails."""
    return rz_shower(seed, nr, nz, n_steps, n_obs, bc=bc, sigma_r=0.02, zmax_frac=(0.15, 0.25),
                     length_range=(0.3, 0.6), r_range=(0.2, 1.2), name=f"rz-small-{nr}x{nz}-{bc}")


def rz_paper_grid(n: int, seed: int = 22, n_steps: Optional[int] = None, n_obs: int = 64) -> RZWorkload:
    """The paper's (r, z) grid sizes (N^2 for N = 256 ... 8192, 1 cm cells), Mur walls, the
    Greisen shower, 64 observers with R up to 64 m where the grid allows; n_steps defaults to N
    (the paper's total work grows as N^3)."""
    return rz_shower(seed, n, n, n if n_steps is None else n_steps, n_obs,
                     zmax_frac=(0.2, 0.3) if n >= 2048 else (0.3, 0.45),
                     length_range=(3.0, 8.0) if n >= 2048 else (0.3, 0.6),
                     r_range=(min(1.0, 0.05 * n * 0.01), 64.0), name=f"rz-{n}x{n}")


def rz_workload_by_name(name: str, seed: Optional[int] = None) -> RZWorkload:
    if name == "rz-small":
        return rz_small(21 if seed is None else seed)
    if name.startswith("rz-") and name[3:].isdigit():
        return rz_paper_grid(int(name[3:]), 22 if seed is None else seed)
    raise KeyError(name)


def rz_workload_digest(w: RZWorkload) -> str:
    h = hashlib.sha256()
    h.update(json.dumps(w.describe(), sort_keys=True).encode())
    for arr in (w.q_bins, w.obs_rz):
        h.update(np.ascontiguousarray(arr, dtype=np.float64).tobytes())
    for v in (w.dt, w.dr, w.dz, w.z_entry, w.sigma_r, w.sigma_z, w.eps_r, w.sigma):
        h.update(np.float64(v).tobytes())
    return h.hexdigest()
