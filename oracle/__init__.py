"""FP64 CPU oracle for the Yee leapfrog with a moving shower current.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product library never imports, links or calls
anything here, and this package imports nothing from the product (it only reads the
plain fields of a ``Workload`` object handed to it).

The numerics live in ``yee_oracle.c`` (plain C, FP64, OpenMP over z planes); this
module builds it on demand with gcc and wraps it with ctypes and numpy.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "yee_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lock = threading.Lock()
_lib = None

BC = {"pec": 0, "mur1": 1, "cpml": 2}


class OrcCfg(ct.Structure):
    _fields_ = [
        ("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32), ("n_steps", ct.c_int32),
        ("dx", ct.c_double), ("dy", ct.c_double), ("dz", ct.c_double), ("dt", ct.c_double),
        ("eps_r", ct.c_double), ("mu_r", ct.c_double), ("sigma", ct.c_double),
        ("bc", ct.c_int32), ("npml", ct.c_int32),
        ("pml_m", ct.c_double), ("pml_sigma_scale", ct.c_double), ("pml_kappa_max", ct.c_double),
        ("pml_alpha_max", ct.c_double),
        ("src_on", ct.c_int32), ("n_bins", ct.c_int32),
        ("x_axis", ct.c_double), ("y_axis", ct.c_double), ("z_entry", ct.c_double),
        ("t_entry", ct.c_double), ("beta", ct.c_double), ("sigma_r", ct.c_double),
        ("sigma_z", ct.c_double), ("cut_sigmas", ct.c_double),
        ("z_bin0", ct.c_double), ("dz_bin", ct.c_double),
        ("q_bins", ct.POINTER(ct.c_double)),
        ("n_obs", ct.c_int32), ("pad0", ct.c_int32),
        ("obs_xyz", ct.POINTER(ct.c_double)),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE semantics, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=gnu11", "-shared", "-fPIC", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ct.CDLL(_LIB)
            P = ct.POINTER(ct.c_double)
            L.orc_create.restype = ct.c_void_p
            L.orc_create.argtypes = [ct.POINTER(OrcCfg)]
            L.orc_destroy.argtypes = [ct.c_void_p]
            L.orc_last_error.restype = ct.c_char_p
            L.orc_field.restype = P
            L.orc_field.argtypes = [ct.c_void_p, ct.c_int]
            L.orc_step_index.restype = ct.c_int32
            L.orc_step_index.argtypes = [ct.c_void_p]
            L.orc_update_h.argtypes = [ct.c_void_p]
            L.orc_update_e.argtypes = [ct.c_void_p]
            L.orc_sample.argtypes = [ct.c_void_p, P]
            L.orc_step.argtypes = [ct.c_void_p, P]
            L.orc_source_current.argtypes = [ct.c_void_p, ct.c_int32, P]
            L.orc_run.restype = ct.c_int
            L.orc_run.argtypes = [ct.POINTER(OrcCfg), P]
            L.orc_run_eps.restype = ct.c_int
            L.orc_run_eps.argtypes = [ct.POINTER(OrcCfg), P, P]
            L.orc_set_eps_map.restype = ct.c_int
            L.orc_set_eps_map.argtypes = [ct.c_void_p, P]
            L.orc_adjoint.restype = ct.c_int
            L.orc_adjoint.argtypes = [ct.POINTER(OrcCfg), P, P]
            L.orc_threads.restype = ct.c_int
            L.orc_set_threads.argtypes = [ct.c_int]
            for f in ("orc_c0", "orc_mu0", "orc_eps0"):
                getattr(L, f).restype = ct.c_double
            _lib = L
        return _lib


def constants():
    L = lib()
    return {"c0": L.orc_c0(), "mu0": L.orc_mu0(), "eps0": L.orc_eps0()}


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def make_cfg(w, q_bins=None):
    """Translate a workload (any object with the Workload fields) into the C struct.
    Returns (cfg, keepalive) -- keep the second item alive while cfg is in use."""
    q = np.ascontiguousarray(w.q_bins if q_bins is None else q_bins, dtype=np.float64)
    obs = np.ascontiguousarray(w.obs_xyz, dtype=np.float64).reshape(-1, 3)
    c = OrcCfg()
    c.nx, c.ny, c.nz, c.n_steps = w.nx, w.ny, w.nz, w.n_steps
    c.dx, c.dy, c.dz, c.dt = w.dx, w.dy, w.dz, w.dt
    c.eps_r, c.mu_r, c.sigma = w.eps_r, w.mu_r, w.sigma
    c.bc = BC[w.bc]
    c.npml = w.npml
    c.pml_m, c.pml_sigma_scale = w.pml_m, w.pml_sigma_scale
    c.pml_kappa_max, c.pml_alpha_max = w.pml_kappa_max, w.pml_alpha_max
    c.src_on = 1 if w.src_on else 0
    c.n_bins = len(q)
    c.x_axis, c.y_axis, c.z_entry, c.t_entry = w.x_axis, w.y_axis, w.z_entry, w.t_entry
    c.beta, c.sigma_r, c.sigma_z, c.cut_sigmas = w.beta, w.sigma_r, w.sigma_z, w.cut_sigmas
    c.z_bin0, c.dz_bin = w.z_bin0, w.dz_bin
    c.q_bins = _dp(q)
    c.n_obs = obs.shape[0]
    c.obs_xyz = _dp(obs)
    return c, (q, obs)


class State:
    """Stepwise access to the oracle's fields (numpy views of the C arrays)."""

    NAMES = ("ex", "ey", "ez", "hx", "hy", "hz")

    def __init__(self, w, q_bins=None):
        self.w = w
        self._cfg, self._keep = make_cfg(w, q_bins)
        L = lib()
        self._h = L.orc_create(ct.byref(self._cfg))
        if not self._h:
            raise ValueError("oracle rejected the configuration: " + L.orc_last_error().decode())
        shape = (w.nz, w.ny, w.nx)
        self.fields = []
        for c in range(6):
            p = L.orc_field(self._h, c)
            self.fields.append(np.ctypeslib.as_array(p, shape=shape))
        self.n_obs = self._cfg.n_obs

    def __getattr__(self, name):
        if name in State.NAMES:
            return self.fields[State.NAMES.index(name)]
        raise AttributeError(name)

    @property
    def n(self) -> int:
        return lib().orc_step_index(self._h)

    def update_h(self):
        lib().orc_update_h(self._h)

    def update_e(self):
        lib().orc_update_e(self._h)

    def sample(self) -> np.ndarray:
        w = np.zeros(3 * max(self.n_obs, 1))
        lib().orc_sample(self._h, _dp(w))
        return w[: 3 * self.n_obs].reshape(self.n_obs, 3)

    def set_eps_map(self, eps_r_map):
        """Per-E-node relative permittivity [3][nz][ny][nx] (None: the uniform medium)."""
        if eps_r_map is None:
            lib().orc_set_eps_map(self._h, None)
            return
        m = np.ascontiguousarray(eps_r_map, dtype=np.float64)
        assert m.shape == (3, self.w.nz, self.w.ny, self.w.nx)
        if lib().orc_set_eps_map(self._h, _dp(m)) != 0:
            raise ValueError("oracle rejected the map: " + lib().orc_last_error().decode())

    def step(self, k: int = 1):
        for _ in range(k):
            lib().orc_step(self._h, None)

    def source_current(self, n: int) -> np.ndarray:
        out = np.zeros((self.w.nz, self.w.ny, self.w.nx))
        lib().orc_source_current(self._h, n, _dp(out))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None
            self.fields = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run(w, q_bins=None) -> np.ndarray:
    """Full forward run from zero fields.  Returns waveforms [n_obs][3][n_steps] (FP64);
    index n is E at time (n+1) dt."""
    cfg, keep = make_cfg(w, q_bins)
    out = np.zeros((max(cfg.n_obs, 1), 3, max(w.n_steps, 1)))
    rc = lib().orc_run(ct.byref(cfg), _dp(out))
    if rc != 0:
        raise ValueError("oracle run failed: " + lib().orc_last_error().decode())
    return out[: cfg.n_obs, :, : w.n_steps]


def run_eps(w, eps_r_map, q_bins=None) -> np.ndarray:
    """Forward run in a heterogeneous medium: eps_r_map [3][nz][ny][nx] gives the relative
    permittivity at every E node (Ca, Cb per node; absorber coefficients stay uniform)."""
    cfg, keep = make_cfg(w, q_bins)
    m = np.ascontiguousarray(eps_r_map, dtype=np.float64)
    assert m.shape == (3, w.nz, w.ny, w.nx)
    out = np.zeros((max(cfg.n_obs, 1), 3, max(w.n_steps, 1)))
    rc = lib().orc_run_eps(ct.byref(cfg), _dp(m), _dp(out))
    if rc != 0:
        raise ValueError("oracle run failed: " + lib().orc_last_error().decode())
    return out[: cfg.n_obs, :, : w.n_steps]


def eps_sensitivity(w, dl_dw: np.ndarray, nodes, rel_step: float = 1e-6, q_bins=None) -> np.ndarray:
    """dL/deps_r at single E nodes for L = <dl_dw, w>, by central differences of the FP64
    forward run with the permittivity of that one node moved by +-rel_step*eps_r.
    nodes: iterable of (comp, k, j, i).  Returns FP64 [len(nodes)]."""
    g = np.asarray(dl_dw, dtype=np.float64)
    base = np.full((3, w.nz, w.ny, w.nx), float(w.eps_r))
    h = rel_step * float(w.eps_r)
    out = []
    for node in nodes:
        vals = []
        for sgn in (1.0, -1.0):
            m = base.copy()
            m[tuple(node)] += sgn * h
            vals.append(float(np.sum(g * run_eps(w, m, q_bins))))
        out.append((vals[0] - vals[1]) / (2.0 * h))
    return np.asarray(out)


def adjoint(w, dl_dw: np.ndarray, q_bins=None) -> np.ndarray:
    """Exact discrete-adjoint gradient dL/dq for a given dL/dw [n_obs][3][n_steps]."""
    cfg, keep = make_cfg(w, q_bins)
    g = np.ascontiguousarray(dl_dw, dtype=np.float64)
    assert g.shape == (cfg.n_obs, 3, w.n_steps)
    out = np.zeros(cfg.n_bins)
    rc = lib().orc_adjoint(ct.byref(cfg), _dp(g), _dp(out))
    if rc != 0:
        raise ValueError("oracle adjoint failed: " + lib().orc_last_error().decode())
    return out
