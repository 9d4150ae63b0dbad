"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

A ctypes wrapper around ``psc_oracle.c``: a plain, slow, obviously-correct FP64
implementation of the partially-saturated-cell LBM step and the JKR DEM step of
Liu & Wu (arXiv 1901.09745), written from the paper (Secs. 2.1-2.5, Eqs. 1-27,
Table 1).  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import it.  It shares no code with the HIP library.

Every function's docstring names the passage it follows.  Nothing here is
"parity unpinned" except the absolute drag of a disk (no closed form) and
long-horizon DEM trajectories (chaotic); the CPU tests pin the rest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "psc_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

KMAX = 16
_FACE = {"periodic": 0, "bounce_back": 1, "moving_wall": 2, "inlet_eq": 3, "outlet_eq": 4}


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc: FP64, no fast-math, no FMA contraction,
    OpenMP over cells."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-D_DEFAULT_SOURCE", "-o", _SO + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)
    return _SO


class _Config(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("tau", ctypes.c_double),
                ("force", ctypes.c_double * 3), ("face_bc", ctypes.c_int * 6),
                ("face_u", (ctypes.c_double * 3) * 6), ("rho0", ctypes.c_double),
                ("h", ctypes.c_double)]


class _Dem(ctypes.Structure):
    _fields_ = [("rho_p", ctypes.c_double), ("rho_f", ctypes.c_double),
                ("E_p", ctypes.c_double), ("poisson", ctypes.c_double),
                ("gamma", ctypes.c_double), ("eta_n", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("dt", ctypes.c_double),
                ("n_sub", ctypes.c_int), ("kinematic", ctypes.c_int),
                ("k_t", ctypes.c_double), ("eta_t", ctypes.c_double),
                ("mu_f", ctypes.c_double), ("theta_r", ctypes.c_double)]


_lib_handle = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        L.or_va2d.restype = ctypes.c_double
        L.or_va2d.argtypes = [ctypes.c_double]
        L.or_va3d.restype = ctypes.c_double
        L.or_va3d.argtypes = [ctypes.c_double]
        L.or_rasterize.argtypes = [ctypes.POINTER(_Config), ctypes.c_int, _D, _D, ctypes.c_int,
                                   _I, _I, _D, _D]
        L.or_feq.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D]
        L.or_guo.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D, _D]
        L.or_moments.argtypes = [ctypes.c_int, _D, _D, _D, _D]
        L.or_omega_s.argtypes = [ctypes.c_int, _D, ctypes.c_double, _D, _D, _D]
        L.or_weights.argtypes = [ctypes.c_int, _D, ctypes.c_double, ctypes.c_int, _D, _D]
        L.or_lbm_step.argtypes = [ctypes.POINTER(_Config), ctypes.c_int, _D, ctypes.c_int,
                                  _D, _D, _D, _D, _D, _D]
        L.or_set_equilibrium.argtypes = [ctypes.POINTER(_Config), _D, _D, _D]
        L.or_macros.argtypes = [ctypes.POINTER(_Config), _D, _D, _D]
        L.or_mass.restype = ctypes.c_double
        L.or_mass.argtypes = [ctypes.POINTER(_Config), _D]
        L.or_jkr_x.restype = ctypes.c_double
        L.or_jkr_x.argtypes = [ctypes.c_double]
        L.or_jkr_force.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, _D, _D]
        L.or_dem_step.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(_Dem), ctypes.c_int,
                                  _D, _D, _D, _D, _D, _D, ctypes.c_int, _I, _I, _D]
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_num_threads.argtypes = [ctypes.c_int]
        _lib_handle = L
    return _lib_handle


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_I)


def _vec(v) -> np.ndarray:
    out = np.zeros(3)
    v = np.asarray(v, dtype=np.float64).ravel()
    out[: v.size] = v
    return out


def make_config(lat) -> _Config:
    """Build the oracle's config from a ``workloads.LatticeSpec``."""
    c = _Config()
    c.q, c.nx, c.ny, c.nz = lat.q, lat.nx, lat.ny, lat.nz
    c.tau = lat.tau
    for a in range(3):
        c.force[a] = lat.force[a]
    for f in range(6):
        c.face_bc[f] = _FACE[lat.faces[f]]
        for a in range(3):
            c.face_u[f][a] = lat.face_u[f][a]
    c.rho0 = lat.rho0
    c.h = lat.h
    return c


def num_threads() -> int:
    return int(_lib().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the OpenMP cell loop (timing only)."""
    _lib().or_set_num_threads(int(n))


# --------------------------------------------------------------------------
# Sec. 2.4: solid fraction
# --------------------------------------------------------------------------

def va2d(r: float) -> float:
    """Eq. 19."""
    return float(_lib().or_va2d(r))


def va3d(r: float) -> float:
    """Eq. 17."""
    return float(_lib().or_va3d(r))


def rasterize(lat, x: np.ndarray, r: np.ndarray, kmax: int = KMAX):
    """Table 1 over all particles.  Returns (nslot[N], ids[N,kmax], eps[N,kmax],
    eps_sum[N]) with cells in canonical order (x fastest); slots in ascending
    particle id."""
    c = make_config(lat)
    N = lat.ncells
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    r = np.ascontiguousarray(r, dtype=np.float64).ravel()
    nslot = np.zeros(N, dtype=np.int32)
    ids = np.full(N * kmax, -1, dtype=np.int32)
    eps = np.zeros(N * kmax)
    ssum = np.zeros(N)
    rc = _lib().or_rasterize(ctypes.byref(c), r.size, _dp(x), _dp(r), kmax, _ip(nslot),
                             _ip(ids), _dp(eps), _dp(ssum))
    if rc:
        raise RuntimeError(f"oracle rasterize failed: {rc}")
    return nslot, ids.reshape(N, kmax), eps.reshape(N, kmax), ssum


# --------------------------------------------------------------------------
# Sec. 2.1 / 2.3 per-cell building blocks
# --------------------------------------------------------------------------

def feq(q: int, rho: float, u) -> np.ndarray:
    """Eq. 3."""
    out = np.zeros(q)
    _lib().or_feq(q, rho, _dp(_vec(u)), _dp(out))
    return out


def guo(q: int, tau: float, u, F) -> np.ndarray:
    """Eq. 4."""
    out = np.zeros(q)
    _lib().or_guo(q, tau, _dp(_vec(u)), _dp(_vec(F)), _dp(out))
    return out


def moments(q: int, f: np.ndarray, F) -> Tuple[float, np.ndarray]:
    """Eq. 5."""
    rho = np.zeros(1)
    u = np.zeros(3)
    _lib().or_moments(q, _dp(np.ascontiguousarray(f, dtype=np.float64)), _dp(_vec(F)),
                      _dp(rho), _dp(u))
    return float(rho[0]), u


def omega_s(q: int, f: np.ndarray, rho: float, u, us) -> np.ndarray:
    """Eq. 10."""
    out = np.zeros(q)
    _lib().or_omega_s(q, _dp(np.ascontiguousarray(f, dtype=np.float64)), rho, _dp(_vec(u)),
                      _dp(_vec(us)), _dp(out))
    return out


def weights(eps, tau: float, mode: int = 0) -> Tuple[float, np.ndarray]:
    """Eq. 13 with the cell total clamped at one (Table 1; mode 0, modified) or Eqs. 8-9 (mode 1,
    original).  Returns (B_n, B_{n,s})."""
    eps = np.ascontiguousarray(eps, dtype=np.float64).ravel()
    Bt = np.zeros(1)
    Bs = np.zeros(max(1, eps.size))
    _lib().or_weights(eps.size, _dp(eps), tau, mode, _dp(Bt), _dp(Bs))
    return float(Bt[0]), Bs[: eps.size]


# --------------------------------------------------------------------------
# Lattice state and steps
# --------------------------------------------------------------------------

class Lattice:
    """Natural-layout FP64 state f[Q, nz, ny, nx] with the oracle's step."""

    def __init__(self, lat, f: Optional[np.ndarray] = None):
        self.spec = lat
        self.cfg = make_config(lat)
        if f is None:
            self.f = np.zeros((lat.q,) + lat.shape)
            self.set_equilibrium()
        else:
            self.f = np.ascontiguousarray(f, dtype=np.float64).reshape((lat.q,) + lat.shape).copy()

    def set_equilibrium(self, rho: Optional[np.ndarray] = None, u: Optional[np.ndarray] = None):
        """f = f^eq(rho, u) (Eq. 3); defaults rho0 and rest."""
        rp = None if rho is None else _dp(np.ascontiguousarray(rho, dtype=np.float64).ravel())
        up = None if u is None else _dp(np.ascontiguousarray(u, dtype=np.float64).reshape(-1))
        _lib().or_set_equilibrium(ctypes.byref(self.cfg), _dp(self.f), rp, up)

    def step(self, p=None, mode: int = 0) -> Tuple[np.ndarray, np.ndarray]:
        """One PSC-LBM step (Eqs. 1, 5-6, 10, 12-14 and Table 1).  Returns the
        per-particle hydrodynamic force and torque (n, 3) of Eq. 14."""
        if p is None or p.n == 0:
            z = np.zeros((1, 3))
            x = u = w = z
            r = np.ones(1)
            n = 0
        else:
            x, u, w, r, n = p.x, p.u, p.omega, p.r, p.n
        F = np.zeros((max(n, 1), 3))
        T = np.zeros((max(n, 1), 3))
        rc = _lib().or_lbm_step(ctypes.byref(self.cfg), mode, _dp(self.f), n,
                                _dp(np.ascontiguousarray(x, dtype=np.float64)),
                                _dp(np.ascontiguousarray(u, dtype=np.float64)),
                                _dp(np.ascontiguousarray(w, dtype=np.float64)),
                                _dp(np.ascontiguousarray(r, dtype=np.float64)), _dp(F), _dp(T))
        if rc:
            raise RuntimeError(f"oracle step failed: {rc}")
        return F[:n], T[:n]

    def macros(self) -> Tuple[np.ndarray, np.ndarray]:
        """(rho[nz,ny,nx], u[nz,ny,nx,3]) by Eq. 5."""
        N = self.spec.ncells
        rho = np.zeros(N)
        u = np.zeros(N * 3)
        _lib().or_macros(ctypes.byref(self.cfg), _dp(self.f), _dp(rho), _dp(u))
        return rho.reshape(self.spec.shape), u.reshape(self.spec.shape + (3,))

    def mass(self) -> float:
        return float(_lib().or_mass(ctypes.byref(self.cfg), _dp(self.f)))


# --------------------------------------------------------------------------
# Sec. 2.5: JKR contact and DEM
# --------------------------------------------------------------------------

def jkr_x(dn: float) -> float:
    """a/a0 on the stable JKR branch for delta/delta_C = dn >= -1."""
    return float(_lib().or_jkr_x(dn))


def jkr_force(R: float, E: float, gamma: float, delta: float) -> Tuple[float, float]:
    """(F_n, delta_C) of Eqs. 26-27 without damping; repulsive positive."""
    F = np.zeros(1)
    dC = np.zeros(1)
    _lib().or_jkr_force(R, E, gamma, delta, _dp(F), _dp(dC))
    return float(F[0]), float(dC[0])


def make_dem(d) -> _Dem:
    p = _Dem()
    p.rho_p, p.rho_f, p.E_p, p.poisson = d.rho_p, d.rho_f, d.E_p, d.poisson
    p.gamma, p.eta_n = d.gamma, d.eta_n
    for a in range(3):
        p.g[a] = d.g[a]
    p.dt, p.n_sub, p.kinematic = d.dt, d.n_sub, int(d.kinematic)
    p.k_t, p.eta_t, p.mu_f, p.theta_r = d.k_t, d.eta_t, d.mu_f, d.theta_r
    return p


class Dem:
    """DEM state (contact history) and the oracle's DEM step (Eq. 21)."""

    def __init__(self, lat, dem, n: int):
        self.cfg = make_config(lat)
        self.params = make_dem(dem)
        self.cap = dem.max_contacts
        self.ncontact = np.zeros(max(n, 1), dtype=np.int32)
        self.ids = np.zeros(max(n, 1) * self.cap, dtype=np.int32)
        # each contact's springs (tangential displacement xi[3], twist angle,
        # rolling displacement xr[3], unused)
        self.hist = np.zeros(max(n, 1) * self.cap * 8)

    def step(self, p, F: np.ndarray, T: np.ndarray) -> None:
        """Advance p in place by one coupling step with fluid force F, torque T."""
        Fc = np.ascontiguousarray(F, dtype=np.float64)
        Tc = np.ascontiguousarray(T, dtype=np.float64)
        rc = _lib().or_dem_step(ctypes.byref(self.cfg), ctypes.byref(self.params), p.n,
                                _dp(p.x), _dp(p.u), _dp(p.omega), _dp(p.r), _dp(Fc), _dp(Tc),
                                self.cap, _ip(self.ncontact), _ip(self.ids), _dp(self.hist))
        if rc:
            raise RuntimeError(f"oracle DEM step failed: {rc}")

    def contacts(self):
        return [sorted(self.ids[i * self.cap: i * self.cap + self.ncontact[i]].tolist())
                for i in range(self.ncontact.size)]

    def springs(self, i: int) -> dict:
        """{contact id: (xi[3], theta, xr[3])} of particle i's contacts."""
        out = {}
        for k in range(self.ncontact[i]):
            h = self.hist[(i * self.cap + k) * 8:(i * self.cap + k + 1) * 8]
            out[int(self.ids[i * self.cap + k])] = (h[:3].copy(), float(h[3]), h[4:7].copy())
        return out
