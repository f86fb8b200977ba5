"""Second, independent FP64 implementation of the discrete scheme, for tiny grids.

TEST INFRASTRUCTURE ONLY: it exists to cross-check the C oracle (tests/test_oracle_pins.py).
It is written separately from the C code -- whole-array NumPy updates instead of loops,
full-size CPML memory arrays instead of slabs, its own source and observer code -- from the
same statement of the method:

- Maxwell's curl equations with conductivity (Numerical Method section), central differences
  on the Yee lattice, leapfrog in time: H^{n+1/2} = H^{n-1/2} - (dt/mu) curl E^n (forward
  differences), E^{n+1} = Ca E^n + Cb (curl H^{n+1/2} - J^{n+1/2}) (backward differences);
- the moving charge-excess current of the Simulation Setup section, J_z = v Q(z_s) W_r W_z with
  discretely normalised Gaussian weights and the bunch centre z_s at (n+1/2) dt;
- PEC walls, first-order Mur on the face-interior tangential E, or a CFS-CPML (psi <- b psi +
  a d, stretched derivative d/kappa + psi);
- E recorded at detector points by trilinear interpolation on each component's sub-lattice.

Conventions: N nodes per axis, walls on node planes 0 and N-1; arrays [z, y, x].
"""
from __future__ import annotations

import math

import numpy as np

C0 = 299_792_458.0
MU0 = 1.25663706212e-6  # CODATA 2018
EPS0 = 1.0 / (MU0 * C0 * C0)


def _grading(w, n: int, delta: float):
    """CPML coefficient profiles along one axis at integer and half-integer positions.
    Returns dicts with arrays a, b, kappa and a boolean 'in' mask, for 'e' (positions i) and
    'h' (positions i + 1/2, i <= n - 2)."""
    npml = w.npml if w.bc == "cpml" else 0
    out = {}
    for kind, offset, count in (("e", 0.0, n), ("h", 0.5, n - 1)):
        pos = np.arange(count) + offset
        depth = np.maximum(np.maximum(npml - pos, pos - (n - 1 - npml)), 0.0) if npml > 0 else np.zeros(count)
        inside = depth > 0.0
        rho = depth / npml if npml > 0 else depth
        sig_opt = 0.8 * (w.pml_m + 1.0) / (MU0 * C0 * delta * math.sqrt(w.eps_r * w.mu_r))
        sigma = w.pml_sigma_scale * sig_opt * rho ** w.pml_m
        kappa = 1.0 + (w.pml_kappa_max - 1.0) * rho ** w.pml_m
        alpha = w.pml_alpha_max * (1.0 - rho)
        b = np.exp(-(sigma / kappa + alpha) * w.dt / EPS0)
        with np.errstate(invalid="ignore", divide="ignore"):
            a = np.where(inside, sigma * (b - 1.0) / (sigma * kappa + kappa * kappa * alpha), 0.0)
        out[kind] = {"a": np.where(inside, a, 0.0), "b": np.where(inside, b, 1.0),
                     "kappa": np.where(inside, kappa, 1.0), "in": inside}
    return out


class NumpyYee:
    """State of one run; step() advances one Yee step and returns E^{n+1} at the observers."""

    def __init__(self, w, q_bins=None):
        self.w = w
        self.q = np.asarray(w.q_bins if q_bins is None else q_bins, dtype=np.float64)
        nx, ny, nz = w.nx, w.ny, w.nz
        shape = (nz, ny, nx)
        self.E = [np.zeros(shape) for _ in range(3)]
        self.H = [np.zeros(shape) for _ in range(3)]
        eps, mu = EPS0 * w.eps_r, MU0 * w.mu_r
        loss = w.sigma * w.dt / (2.0 * eps)
        self.ca = (1.0 - loss) / (1.0 + loss)
        self.cb = (w.dt / eps) / (1.0 + loss)
        self.db = w.dt / mu
        self.g = [_grading(w, n, d) for n, d in ((nx, w.dx), (ny, w.dy), (nz, w.dz))]
        # psi for (field, derivative axis), full arrays (zero outside the layers)
        self.psi_h = {key: np.zeros(shape) for key in ("xy", "xz", "yz", "yx", "zx", "zy")}
        self.psi_e = {key: np.zeros(shape) for key in ("xy", "xz", "yz", "yx", "zx", "zy")}
        self.n = 0
        self._source_tables()
        self._observer_tables()

    # -- source
    def _source_tables(self):
        w = self.w
        self.wr = np.zeros((w.ny, w.nx))
        if not w.src_on:
            return
        jj, ii = np.meshgrid(np.arange(w.ny), np.arange(w.nx), indexing="ij")
        r2 = (ii * w.dx - w.x_axis) ** 2 + (jj * w.dy - w.y_axis) ** 2
        nodes = (ii >= 1) & (ii <= w.nx - 2) & (jj >= 1) & (jj <= w.ny - 2) & (r2 <= (w.cut_sigmas * w.sigma_r) ** 2)
        g = np.where(nodes, np.exp(-0.5 * r2 / w.sigma_r ** 2), 0.0)
        self.wr = g / (g.sum() * w.dx * w.dy)

    def charge(self, z: float) -> float:
        """Q(z): hat-function interpolation of the profile bins (zero outside them)."""
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
        """J_z on the Ez lattice at time (n + 1/2) dt."""
        w = self.w
        jz = np.zeros((w.nz, w.ny, w.nx))
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
        jz[ks[keep]] = v * self.charge(zs) * wz[keep][:, None, None] * self.wr[None]
        return jz

    # -- observers
    def _observer_tables(self):
        w = self.w
        d = (w.dx, w.dy, w.dz)
        self.stencils = []
        for o in np.asarray(w.obs_xyz, dtype=np.float64).reshape(-1, 3):
            per_comp = []
            for c in range(3):
                base, frac = [], []
                for u in range(3):
                    f = o[u] / d[u] - (0.5 if u == c else 0.0)
                    base.append(int(math.floor(f)))
                    frac.append(f - math.floor(f))
                per_comp.append((base, frac))
            self.stencils.append(per_comp)

    def sample(self) -> np.ndarray:
        out = np.zeros((len(self.stencils), 3))
        for o, per_comp in enumerate(self.stencils):
            for c, (b, t) in enumerate(per_comp):
                cube = self.E[c][b[2]:b[2] + 2, b[1]:b[1] + 2, b[0]:b[0] + 2]
                wx = np.array([1.0 - t[0], t[0]])
                wy = np.array([1.0 - t[1], t[1]])
                wz = np.array([1.0 - t[2], t[2]])
                out[o, c] = np.einsum("kji,k,j,i->", cube, wz, wy, wx)
        return out

    # -- stretched derivative: d/kappa + psi (psi updated) inside the layer, d elsewhere
    def _stretch(self, psi, d, axis: int, kind: str, sl):
        g = self.g[axis][kind]
        shape = [1, 1, 1]
        shape[2 - axis] = -1
        a = g["a"][sl].reshape(shape)
        b = g["b"][sl].reshape(shape)
        k = g["kappa"][sl].reshape(shape)
        m = g["in"][sl].reshape(shape)
        new = np.where(m, b * psi + a * d, 0.0)
        psi[...] = new
        return np.where(m, d / k + new, d)

    def update_h(self):
        w = self.w
        ex, ey, ez = self.E
        hx, hy, hz = self.H
        s = slice(None)
        # Hx(i, j+1/2, k+1/2): k, j <= n-2
        dy_ez = (ez[:-1, 1:, :] - ez[:-1, :-1, :]) / w.dy
        dz_ey = (ey[1:, :-1, :] - ey[:-1, :-1, :]) / w.dz
        ty = self._stretch(self.psi_h["xy"][:-1, :-1, :], dy_ez, 1, "h", slice(0, w.ny - 1))
        tz = self._stretch(self.psi_h["xz"][:-1, :-1, :], dz_ey, 2, "h", slice(0, w.nz - 1))
        hx[:-1, :-1, :] -= self.db * (ty - tz)
        # Hy(i+1/2, j, k+1/2): k, i <= n-2
        dz_ex = (ex[1:, :, :-1] - ex[:-1, :, :-1]) / w.dz
        dx_ez = (ez[:-1, :, 1:] - ez[:-1, :, :-1]) / w.dx
        tz = self._stretch(self.psi_h["yz"][:-1, :, :-1], dz_ex, 2, "h", slice(0, w.nz - 1))
        tx = self._stretch(self.psi_h["yx"][:-1, :, :-1], dx_ez, 0, "h", slice(0, w.nx - 1))
        hy[:-1, :, :-1] -= self.db * (tz - tx)
        # Hz(i+1/2, j+1/2, k): j, i <= n-2
        dx_ey = (ey[:, :-1, 1:] - ey[:, :-1, :-1]) / w.dx
        dy_ex = (ex[:, 1:, :-1] - ex[:, :-1, :-1]) / w.dy
        tx = self._stretch(self.psi_h["zx"][:, :-1, :-1], dx_ey, 0, "h", slice(0, w.nx - 1))
        ty = self._stretch(self.psi_h["zy"][:, :-1, :-1], dy_ex, 1, "h", slice(0, w.ny - 1))
        hz[:, :-1, :-1] -= self.db * (tx - ty)
        del s

    def update_e(self):
        w = self.w
        ex, ey, ez = self.E
        hx, hy, hz = self.H
        old = [e.copy() for e in self.E] if w.bc == "mur1" else None
        jz = self.current_z(self.n)
        I = slice(1, w.nx - 1)
        J = slice(1, w.ny - 1)
        K = slice(1, w.nz - 1)
        # Ex(i+1/2, j, k): i <= nx-2, 1 <= j, k <= n-2
        dy_hz = (hz[K, J, :-1] - hz[K, 0:w.ny - 2, :-1]) / w.dy
        dz_hy = (hy[K, J, :-1] - hy[0:w.nz - 2, J, :-1]) / w.dz
        ty = self._stretch(self.psi_e["xy"][K, J, :-1], dy_hz, 1, "e", J)
        tz = self._stretch(self.psi_e["xz"][K, J, :-1], dz_hy, 2, "e", K)
        ex[K, J, :-1] = self.ca * ex[K, J, :-1] + self.cb * (ty - tz)
        # Ey(i, j+1/2, k): 1 <= i <= nx-2, j <= ny-2, 1 <= k <= nz-2
        dz_hx = (hx[K, :-1, I] - hx[0:w.nz - 2, :-1, I]) / w.dz
        dx_hz = (hz[K, :-1, I] - hz[K, :-1, 0:w.nx - 2]) / w.dx
        tz = self._stretch(self.psi_e["yz"][K, :-1, I], dz_hx, 2, "e", K)
        tx = self._stretch(self.psi_e["yx"][K, :-1, I], dx_hz, 0, "e", I)
        ey[K, :-1, I] = self.ca * ey[K, :-1, I] + self.cb * (tz - tx)
        # Ez(i, j, k+1/2): 1 <= i, j <= n-2, k <= nz-2
        dx_hy = (hy[:-1, J, I] - hy[:-1, J, 0:w.nx - 2]) / w.dx
        dy_hx = (hx[:-1, J, I] - hx[:-1, 0:w.ny - 2, I]) / w.dy
        tx = self._stretch(self.psi_e["zx"][:-1, J, I], dx_hy, 0, "e", I)
        ty = self._stretch(self.psi_e["zy"][:-1, J, I], dy_hx, 1, "e", J)
        ez[:-1, J, I] = self.ca * ez[:-1, J, I] + self.cb * (tx - ty - jz[:-1, J, I])
        if old is not None:
            self._mur(old)
        self.n += 1

    def _mur(self, old):
        """First-order Mur on the face-interior tangential E (edges held at zero)."""
        w = self.w
        v = C0 / math.sqrt(w.eps_r * w.mu_r)
        ex, ey, ez = self.E
        ox, oy, oz = old

        def k(d):
            return (v * w.dt - d) / (v * w.dt + d)

        kx, ky, kz = k(w.dx), k(w.dy), k(w.dz)
        nx, ny, nz = w.nx, w.ny, w.nz
        # x faces: Ey (j <= ny-2, 1 <= k <= nz-2), Ez (1 <= j <= ny-2, k <= nz-2)
        for f, o, ks, js in ((ey, oy, slice(1, nz - 1), slice(0, ny - 1)), (ez, oz, slice(0, nz - 1), slice(1, ny - 1))):
            f[ks, js, 0] = o[ks, js, 1] + kx * (f[ks, js, 1] - o[ks, js, 0])
            f[ks, js, nx - 1] = o[ks, js, nx - 2] + kx * (f[ks, js, nx - 2] - o[ks, js, nx - 1])
        # y faces: Ex (i <= nx-2, 1 <= k <= nz-2), Ez (1 <= i <= nx-2, k <= nz-2)
        for f, o, ks, is_ in ((ex, ox, slice(1, nz - 1), slice(0, nx - 1)), (ez, oz, slice(0, nz - 1), slice(1, nx - 1))):
            f[ks, 0, is_] = o[ks, 1, is_] + ky * (f[ks, 1, is_] - o[ks, 0, is_])
            f[ks, ny - 1, is_] = o[ks, ny - 2, is_] + ky * (f[ks, ny - 2, is_] - o[ks, ny - 1, is_])
        # z faces: Ex (1 <= j <= ny-2, i <= nx-2), Ey (j <= ny-2, 1 <= i <= nx-2)
        for f, o, js, is_ in ((ex, ox, slice(1, ny - 1), slice(0, nx - 1)), (ey, oy, slice(0, ny - 1), slice(1, nx - 1))):
            f[0, js, is_] = o[1, js, is_] + kz * (f[1, js, is_] - o[0, js, is_])
            f[nz - 1, js, is_] = o[nz - 2, js, is_] + kz * (f[nz - 2, js, is_] - o[nz - 1, js, is_])

    def step(self) -> np.ndarray:
        self.update_h()
        self.update_e()
        return self.sample()


def run(w, q_bins=None) -> np.ndarray:
    """Waveforms [n_obs][3][n_steps]; column n is E at (n+1) dt."""
    st = NumpyYee(w, q_bins)
    out = np.zeros((len(st.stencils), 3, w.n_steps))
    for n in range(w.n_steps):
        out[:, :, n] = st.step()
    return out
